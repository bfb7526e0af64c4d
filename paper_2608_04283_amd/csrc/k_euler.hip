// Kernels of one hyperbolic system; see vklb_system.inc.
#define VKLB_KIND vklb::K_EULER
#define VKLB_NAME launchers_euler
#include "vklb_system.inc"
