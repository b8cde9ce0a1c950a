// The analysis kernel for workgroups of 257..1024 threads: the same device
// code as ig_kernels.hip, compiled in a translation unit of its own so that
// its register budget (128 per lane at 1024 threads) does not constrain the
// 256-thread build.
#define IG_WIDE_ONLY 1
#include "ig_kernels.hip"
