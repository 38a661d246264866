// srwcr_lbfgs.cpp -- multi-resolution L-BFGS registration driver (Sec. II-F).
#include <hip/hip_runtime.h>

#include "srwcr.h"

extern "C" int register_lbfgs(const srwcr_problem *prob, const float *fixed, const float *moving, float *ffd_inout,
                              const srwcr_lbfgs_opts *opts, srwcr_lbfgs_report *report, void *stream)
{
    (void)prob; (void)fixed; (void)moving; (void)ffd_inout; (void)opts; (void)report; (void)stream;
    return SRWCR_E_UNSUPPORTED;
}
