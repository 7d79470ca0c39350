// One instantiation of the stitch kernel: block size TK_NTT threads, trees of
// at most TK_PM modes (the build compiles this file once per pair, in
// parallel), with its launcher, its LDS limit and its occupancy query.
#include "tk_stitch.hpp"

#if !defined(TK_NTT) || !defined(TK_PM)
#error "compile with -DTK_NTT=<64|128|256> -DTK_PM=<4|7>"
#endif

#define TK_CAT2_(a, b, c) a##b##_##c
#define TK_CAT_(a, b, c) TK_CAT2_(a, b, c)
#define TK_ENTRY(name) TK_CAT_(name, TK_NTT, TK_PM)

namespace tk {

static_assert(TK_PM == PM_FEW || TK_PM == MAXP, "stitch instantiations hold up to four or up to MAXP modes");

hipError_t TK_ENTRY(stitch_launch_)(const StitchArgs& a, int grid, size_t lds_bytes, hipStream_t stream) {
  hipLaunchKernelGGL((stitch_kernel<TK_NTT, TK_PM>), dim3(grid), dim3(TK_NTT), lds_bytes, stream, a);
  return hipGetLastError();
}

hipError_t TK_ENTRY(stitch_set_lds_)(size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(stitch_kernel<TK_NTT, TK_PM>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

int TK_ENTRY(stitch_occupancy_)(size_t lds_bytes) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stitch_kernel<TK_NTT, TK_PM>, TK_NTT, lds_bytes) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

}  // namespace tk
