// hg_render_mfma.hip -- mixed-precision forward (placeholder until the
// matrix-core kernel lands).
#include "hg_launch.h"

namespace hg {
hipError_t launch_render_mixed(const RenderK &, bool, bool, hipStream_t) { return hipErrorNotSupported; }
}  // namespace hg
