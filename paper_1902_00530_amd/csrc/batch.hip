// Batched sweeps over many lattices (placeholder until the batched kernel lands).
#include "internal.h"

using namespace lbm;

extern "C" {

size_t lbm_sweep_workspace_bytes(const lbm_params *ps, int32_t n)
{
    (void)ps;
    (void)n;
    return 0;
}

int32_t lbm_sweep_batch(const lbm_params *ps, int32_t n, const lbm_sweep_opts *o, void *const *bufs, void *ws,
                        size_t ws_bytes, void *stream, lbm_obs *out)
{
    (void)ps; (void)n; (void)o; (void)bufs; (void)ws; (void)ws_bytes; (void)stream; (void)out;
    return fail(LBM_EUNSUPPORTED, "lbm_sweep_batch not built yet");
}

}
