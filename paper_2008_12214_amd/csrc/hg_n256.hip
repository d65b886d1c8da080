// Kernels and launchers for transform length 256.
#define HG_N 256
#include "hg_sizes.inc"
