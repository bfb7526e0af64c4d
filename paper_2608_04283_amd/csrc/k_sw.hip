// Kernels of one hyperbolic system; see vklb_system.inc.
#define VKLB_KIND vklb::K_SW
#define VKLB_NAME launchers_sw
#include "vklb_system.inc"
