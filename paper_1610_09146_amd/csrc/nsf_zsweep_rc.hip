// The recompute-all form of the z-marching kernels (RA: residual, fused
// stage, batched stage; paper Section 2) in a translation unit of its own:
// the kernel templates of nsf_zsweep.hip instantiated with RC = true and no
// stored gradients, and the launch functions the main unit calls for them.
// Built with the default scheduler setting (see build.py).
#define NSF_ZSWEEP_RC_UNIT 1
#include "nsf_zsweep.hip"
