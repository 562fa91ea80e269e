"""MI355X-native switched-Hamiltonian molecular dynamics for silicon.

Hot path of non-equilibrium free-energy and dynamic Clausius-Clapeyron
integration runs: cell-list neighbour build, Stillinger-Weber energy / force /
virial, Langevin + isotropic-barostat velocity Verlet, the lambda-switched
Hamiltonian and its work integral.  The compute runs in hand-written HIP
kernels behind the C-ABI library ``libswfe.so``; ``swfe`` is its ctypes
binding.  Importing this package loads nothing: ``inputs`` is plain numpy and
the library is opened on first use of ``swfe``.
"""
