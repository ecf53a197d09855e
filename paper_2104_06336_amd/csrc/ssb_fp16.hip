// FP16 hi+lo split-precision instantiations of the fused scan-DFT kernels (matrix cores).
#include "ssb_fused.h"

namespace stem {

template int launch_xstage_p<STEM_DFT_FP16_SPLIT, uint8_t>(int, const uint8_t*, int, int, int, int64_t, float2*, hipStream_t);
template int launch_xstage_p<STEM_DFT_FP16_SPLIT, uint16_t>(int, const uint16_t*, int, int, int, int64_t, float2*, hipStream_t);
template int launch_yreduce_p<STEM_DFT_FP16_SPLIT>(int, const YArgs&, const Optics&, int, int, hipStream_t);
template int launch_yadjoint_p<STEM_DFT_FP16_SPLIT>(int, const YArgs&, const Optics&, hipStream_t);

}  // namespace stem
