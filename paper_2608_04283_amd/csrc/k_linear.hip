// Kernels of one hyperbolic system; see vklb_system.inc.
#define VKLB_KIND vklb::K_LINEAR
#define VKLB_NAME launchers_linear
#include "vklb_system.inc"
