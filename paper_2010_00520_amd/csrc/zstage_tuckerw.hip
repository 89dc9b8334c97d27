// Kernel instantiations for the Tucker family restored from a formed x-mode
// product (ZF_TUCKER_W1, three-pass path only); compiled separately so the
// families build in parallel.
#include "stages.h"

namespace tfmm {
template hipError_t launch_zstage_fmt<ZF_TUCKER_W1>(const ZArgs&, hipStream_t, bool*);
}  // namespace tfmm
