// Kernels of one hyperbolic system; see vklb_system.inc.
#define VKLB_KIND vklb::K_MHD
#define VKLB_NAME launchers_mhd
#include "vklb_system.inc"
