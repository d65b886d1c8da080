// Kernels and launchers for transform length 4096.
#define HG_N 4096
#include "hg_sizes.inc"
