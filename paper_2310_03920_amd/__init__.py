"""MI355X-native two-site DMRG sigma-vector path (H_eff . psi) for ab initio
Hamiltonians with U(1) x U(1) (N, Sz) block sparsity.

Host layers: `mpo` (NC-partition MPO), `_lib` (ctypes binding of the HIP
library), `dmrg` (two-site sweep driver).  All contractions run in the HIP
library `libheffx.so` built from `csrc/`.
"""
