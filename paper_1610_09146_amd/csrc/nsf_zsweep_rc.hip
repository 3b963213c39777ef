// The recompute forms of the z-marching kernels (RA, and RS over each store
// set; paper Section 2) in a translation unit of their own: the kernel
// templates of nsf_zsweep.hip instantiated with RC = true, and the launch
// functions the main unit calls for them. Built with the default scheduler
// setting (see build.py).
#define NSF_ZSWEEP_RC_UNIT 1
#include "nsf_zsweep.hip"
