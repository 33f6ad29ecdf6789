// Batched launches over independent problems and the continuous-batching
// solve server.  (Filled in below the stubs as the batched kernels land.)
#include "fem_internal.h"
#include "host_api.h"
#include "launch.h"

using namespace fem;

#define NOT_YET(name) return set_error(FEM_EINVAL, name ": not available in this build")

extern "C" fem_status fem_batch_create(int, const fem_desc*, void*, fem_batch** out) {
    if (out) *out = nullptr;
    NOT_YET("fem_batch_create");
}
extern "C" fem_status fem_batch_destroy(fem_batch*) { return FEM_OK; }
extern "C" fem_status fem_batch_problem(fem_batch*, int, fem_problem**) { NOT_YET("fem_batch_problem"); }
extern "C" fem_status fem_batch_apply(fem_batch*, void* const*, void* const*, int) { NOT_YET("fem_batch_apply"); }
extern "C" fem_status fem_batch_patch_inverse(fem_batch*, void* const*, void* const*, int) {
    NOT_YET("fem_batch_patch_inverse");
}
extern "C" fem_status fem_batch_autotune(fem_batch*, int, int*) { NOT_YET("fem_batch_autotune"); }
extern "C" fem_status fem_server_create(size_t, int, int, int, double, void*, fem_server** out) {
    if (out) *out = nullptr;
    NOT_YET("fem_server_create");
}
extern "C" fem_status fem_server_destroy(fem_server*) { return FEM_OK; }
extern "C" fem_status fem_server_submit(fem_server*, const fem_desc*, const double*, double, int, uint64_t*) {
    NOT_YET("fem_server_submit");
}
extern "C" fem_status fem_server_step(fem_server*, int*, int*, int*) { NOT_YET("fem_server_step"); }
extern "C" fem_status fem_server_poll(fem_server*, uint64_t, double*, fem_solve_info*) { NOT_YET("fem_server_poll"); }
extern "C" fem_status fem_server_memory(fem_server*, size_t*, size_t*) { NOT_YET("fem_server_memory"); }
