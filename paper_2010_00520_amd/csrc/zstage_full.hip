// Kernel instantiations for one operator family (ZF_FULL); compiled separately so
// the families build in parallel.
#include "stages.h"

namespace tfmm {
template hipError_t launch_zstage_fmt<ZF_FULL>(const ZArgs&, hipStream_t, bool*);
template hipError_t launch_fused_fmt<ZF_FULL>(const ZArgs&, const RhsPtrs&, float, hipStream_t, bool*);
}  // namespace tfmm
