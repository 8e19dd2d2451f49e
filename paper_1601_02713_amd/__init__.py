"""MI355X-native batched direct-SCF (RHF) energies and forces for replica
simulations.  The compute path is libbeadscf.so (HIP kernels for gfx950) behind
the C ABI in include/beadscf.h; ``beadscf`` is its ctypes binding."""
