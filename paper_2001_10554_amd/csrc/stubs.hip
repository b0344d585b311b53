// Entry points whose kernels are not built yet: they report QS_ERR_UNSUPPORTED.
#include "launch.h"

#define QS_API extern "C" __attribute__((visibility("default")))

QS_API int qs_pool_workspace_bytes(const qs_pool_desc *, size_t *) { return qs::fail(QS_ERR_UNSUPPORTED, "pool not built"); }
QS_API int qs_pool_run(const qs_pool_desc *, const double *, double *, double *, void *, size_t, void *) {
    return qs::fail(QS_ERR_UNSUPPORTED, "pool not built");
}
