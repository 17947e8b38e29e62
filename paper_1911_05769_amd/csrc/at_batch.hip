// Batched 1D form of libat.so (placeholder until the kernel lands).
#include "../../include/at.h"
#include "at_internal.h"

at_status at_fail(at_status st, const char *msg);

extern "C" {
at_status at_batch_workspace_bytes(const at_config *, int32_t, uint64_t *)
{ return at_fail(AT_ERR_ARG, "batched form not built yet"); }
at_status at_batch_init(const at_config *, int32_t, void *, uint64_t, at_batch **)
{ return at_fail(AT_ERR_ARG, "batched form not built yet"); }
void at_batch_free(at_batch *) {}
at_status at_batch_run(at_batch *, double *const *, double *const *, int64_t, int32_t)
{ return at_fail(AT_ERR_ARG, "batched form not built yet"); }
at_status at_batch_autotune(at_batch *, double *const *, double *const *, double *const *,
                            int32_t, int32_t *)
{ return at_fail(AT_ERR_ARG, "batched form not built yet"); }
at_status at_batch_set_fuse(at_batch *, int32_t)
{ return at_fail(AT_ERR_ARG, "batched form not built yet"); }
}
