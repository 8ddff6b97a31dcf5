"""MI355X-native moment-conserving GW: the density-fitted hot path (TDA/RPA
density-response moments, self-energy moments, block-Lanczos poles and the
upfolded Hamiltonian) as HIP kernels for gfx950 behind the C ABI in
include/gwmom.h.  ``gwmom`` is the ctypes binding; ``build`` compiles the
library in-tree.  Importing the package loads nothing."""
