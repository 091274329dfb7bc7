#include "internal.hpp"
using namespace sg;
extern "C" {
sg_status sg_solve_batched_impl(Scene &, const sg_solve_opts &, hipStream_t, double *, int, sg_solve_info *) {
    set_error("batched solve not built yet"); return SG_E_INVALID; }
sg_status sg_server_create(sg_ctx *, const sg_server_opts *, sg_server **) { set_error("no server"); return SG_E_INVALID; }
sg_status sg_submit(sg_server *, const sg_scene_desc *, uint64_t *) { return SG_E_INVALID; }
sg_status sg_poll(sg_server *, uint64_t, double *, sg_solve_info *, int32_t *) { return SG_E_INVALID; }
sg_status sg_wait(sg_server *, uint64_t, double *, sg_solve_info *) { return SG_E_INVALID; }
sg_status sg_server_latencies(sg_server *, double *, int32_t, int32_t *) { return SG_E_INVALID; }
sg_status sg_server_destroy(sg_server *) { return SG_E_INVALID; }
}
