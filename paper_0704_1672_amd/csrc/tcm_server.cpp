// Serving loop of libtcm (continuous batching).  Placeholder until the serving thread lands:
// the entry points validate their arguments and report that no server is running.
#include "tcm_runtime.h"

namespace tcm {
void server_destroy(Ctx* c) { (void)c; }
}  // namespace tcm

extern "C" int tcm_server_start(tcm_ctx* t, const tcm_server_cfg* cfg)
{
    (void)t; (void)cfg;
    return TCM_EINVAL;
}
extern "C" int tcm_submit(tcm_ctx* t, const tcm_request* r, uint64_t* tk)
{
    (void)t; (void)r; (void)tk;
    return TCM_EINVAL;
}
extern "C" int tcm_poll(tcm_ctx* t, uint64_t tk, double* U, int32_t* st, double* lat)
{
    (void)t; (void)tk; (void)U; (void)st; (void)lat;
    return TCM_ENOTFOUND;
}
extern "C" int tcm_server_stop(tcm_ctx* t)
{
    (void)t;
    return TCM_EINVAL;
}
extern "C" int tcm_server_stats(tcm_ctx* t, int64_t* a, int64_t* b, int64_t* c, int64_t* d, int64_t* e)
{
    (void)t; (void)a; (void)b; (void)c; (void)d; (void)e;
    return TCM_EINVAL;
}
