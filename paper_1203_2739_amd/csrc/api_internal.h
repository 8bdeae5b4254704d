// Helpers shared by the translation units that implement the C interface.
#pragma once

#include <hip/hip_runtime.h>

#include <exception>
#include <new>

#include "spx_internal.h"

namespace spx {

void hip_check(hipError_t e, const char *what);

// y <- A x with the plan's binary64 values (split plans: accumulate as in
// spx_spmv_split).
hipError_t run_product(spx_plan_s &P, const double *x, double *y, int32_t accumulate, hipStream_t s);

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
