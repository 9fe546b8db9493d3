// Continuous-batching solve server (entry points; the batched implementation
// follows).
#include <string.h>

#include "runtime.hpp"

using namespace spk;

extern "C" {

void spk_server_opts_default(spk_server_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->hbm_budget_bytes = 8ll << 30;
    o->max_slots = 64;
    o->graph_k = 8;
    o->max_blocks_per_system = 256;
}

int spk_server_create(const spk_server_opts *, void *, spk_server **out)
{
    if (out) *out = nullptr;
    set_error("server not available in this build");
    return SPK_EINVAL;
}

int spk_server_submit(spk_server *, int32_t, int64_t, const int32_t *, const int32_t *,
                      const double *, const double *, const spk_ksp_opts *, uint64_t *)
{
    set_error("server not available in this build");
    return SPK_EINVAL;
}

int spk_server_progress(spk_server *, int32_t)
{
    set_error("server not available in this build");
    return SPK_EINVAL;
}

int spk_server_poll(spk_server *, uint64_t, double *, spk_ksp_result *, double *)
{
    set_error("server not available in this build");
    return SPK_EINVAL;
}

int spk_server_destroy(spk_server *) { return SPK_OK; }

}  // extern "C"
