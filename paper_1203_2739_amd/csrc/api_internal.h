// Helpers shared by the translation units that implement the C interface.
#pragma once

#include <hip/hip_runtime.h>

#include <exception>
#include <new>
#include <vector>

#include "spx_internal.h"

namespace spx {

void hip_check(hipError_t e, const char *what);

// y <- A x with the plan's binary64 values (split plans: accumulate as in
// spx_spmv_split).
hipError_t run_product(spx_plan_s &P, const double *x, double *y, int32_t accumulate, hipStream_t s);
// Low-precision product y <- A_low x (binary32 vectors); the plan must hold
// values of that precision (check_lowp_plan).
hipError_t run_lowp(const spx_plan_s &P, int32_t prec, const float *x, float *y, hipStream_t s);
void check_lowp_plan(const spx_plan_s &P, int32_t prec, bool need_device);
bool lowp_schedule_ok(const Tune &t);
// A plan of form SB, DB or split from a given partition, scheduled with
// `tune` (NULL: default) and uploaded when A is on the device.
spx_plan_s *plan_from_partition(const spx_mat_s &A, int form, int32_t K, const PartitionResult &r,
                                const spx_tune *tune);
// Candidate schedules of spx_plan_autotune, in the order they are tried.
const std::vector<spx_tune> &autotune_candidates();

// Runs f, turning exceptions into a status and the thread's last error.
template <class F>
spx_status guarded(F f) {
    try {
        f();
        return SPX_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return SPX_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return SPX_EINVAL;
    } catch (...) {
        set_last_error("unknown error");
        return SPX_EINVAL;
    }
}

}  // namespace spx
