// Kernels and launchers for transform length 1024.
#define HG_N 1024
#include "hg_sizes.inc"
