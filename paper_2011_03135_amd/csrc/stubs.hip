// Temporary entry points for paths still being written.
#include "gpm_internal.h"
namespace gpm {
gpm_status batch_workspace_bytes(int32_t, int32_t, uint64_t *) { return fail(GPM_UNSUPPORTED, "batch not built yet"); }
gpm_status batch_run(const gpm_graph *, const int32_t *, int32_t, int32_t, void *, uint64_t, unsigned long long *, hipStream_t) { return fail(GPM_UNSUPPORTED, "batch not built yet"); }
}
