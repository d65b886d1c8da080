// Kernels and launchers for transform length 2048.
#define HG_N 2048
#include "hg_sizes.inc"
