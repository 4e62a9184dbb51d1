// Autotuner (placeholder until the timing loop lands).
#include "qd_internal.h"

extern "C" {
int qd_autotune(qd_state*, const char*) { return qd::fail(QD_EINVAL, "autotuner not available"); }
int qd_tune_load(const char*) { return qd::fail(QD_EINVAL, "autotuner not available"); }
}
