// Serving loop: resident geometries and asynchronous deformation requests.
#include "internal.h"

namespace rbf {
class Server {};

void server_shutdown(rbf_ctx ctx)
{
    delete ctx->server;
    ctx->server = nullptr;
}
}  // namespace rbf

using namespace rbf;

extern "C" {

rbf_status rbf_geom_create(rbf_ctx, int32_t, int64_t, const double *, int64_t, const double *,
                           const double *, rbf_geom *)
{
    return fail(RBF_E_INVALID, "serving not available in this build");
}

rbf_status rbf_geom_release(rbf_ctx, rbf_geom) { return fail(RBF_E_NOT_FOUND, "no geometry"); }

rbf_status rbf_submit(rbf_ctx, const rbf_request *, rbf_ticket *)
{
    return fail(RBF_E_INVALID, "serving not available in this build");
}

rbf_status rbf_poll(rbf_ctx, rbf_ticket, rbf_req_info *) { return fail(RBF_E_NOT_FOUND, "no ticket"); }

rbf_status rbf_wait(rbf_ctx, rbf_ticket, rbf_req_info *) { return fail(RBF_E_NOT_FOUND, "no ticket"); }

}  // extern "C"
