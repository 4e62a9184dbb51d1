// Batched circuits (placeholder until the persistent layer kernel lands).
#include "qd_internal.h"

extern "C" {
int qd_batch_create(int32_t, const int32_t*, const int32_t*, int32_t, void*, qd_batch**) { return qd::fail(QD_EINVAL, "batched path not available"); }
int qd_batch_size(const qd_batch*, int64_t*) { return qd::fail(QD_EINVAL, "batched path not available"); }
int qd_batch_offset(const qd_batch*, int32_t, int64_t*) { return qd::fail(QD_EINVAL, "batched path not available"); }
int qd_batch_reset(qd_batch*) { return qd::fail(QD_EINVAL, "batched path not available"); }
int qd_batch_apply_layer(qd_batch*, const qd_gate*) { return qd::fail(QD_EINVAL, "batched path not available"); }
int qd_batch_capture(qd_batch*, int32_t) { return qd::fail(QD_EINVAL, "batched path not available"); }
int qd_batch_replay(qd_batch*) { return qd::fail(QD_EINVAL, "batched path not available"); }
int qd_batch_download(const qd_batch*, void*, int64_t) { return qd::fail(QD_EINVAL, "batched path not available"); }
void qd_batch_free(qd_batch*) {}
}
