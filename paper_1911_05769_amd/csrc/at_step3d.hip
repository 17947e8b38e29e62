// 3D vector stepper of libat.so (placeholder until the kernel lands).
#include "../../include/at.h"
#include "at_internal.h"

at_status at_fail(at_status st, const char *msg);

at_status at3_check(const at_config *c)
{
    (void)c;
    return at_fail(AT_ERR_ARG, "3D stepper not built yet");
}

uint64_t at3_ring_level_doubles(const at_config *c)
{
    (void)c;
    return 0;
}

struct at_ctx;
at_status at3_launch(at_ctx *c, const double *uin, double *uout, int64_t n0, int s, int publish)
{
    (void)c; (void)uin; (void)uout; (void)n0; (void)s; (void)publish;
    return at_fail(AT_ERR_ARG, "3D stepper not built yet");
}

int at3_max_fuse(const at_ctx *c)
{
    (void)c;
    return 1;
}
