// Kernels and launchers for transform length 64.
#define HG_N 64
#include "hg_sizes.inc"
