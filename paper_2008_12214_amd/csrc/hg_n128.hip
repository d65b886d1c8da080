// Kernels and launchers for transform length 128.
#define HG_N 128
#include "hg_sizes.inc"
