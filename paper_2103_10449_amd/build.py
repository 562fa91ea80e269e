"""Build of libswfe.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libswfe.so")
SOURCES = [os.path.join(HERE, "csrc", "swfe_kernels.hip"), os.path.join(HERE, "csrc", "swfe_api.hip")]
HEADERS = [os.path.join(HERE, "csrc", "swfe_internal.h"),
           os.path.join(os.path.dirname(HERE), "include", "swfe.h")]

FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         # packed FP32 instructions stay off: the compiler would form them from FP32 code, and some of
         # their forms have given intermittent wrong results on gfx950
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    """Compile the library; always rebuilds.  Returns its path."""
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
