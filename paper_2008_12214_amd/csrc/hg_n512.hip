// Kernels and launchers for transform length 512.
#define HG_N 512
#include "hg_sizes.inc"
