// Split-precision chi sum (placeholder until the BF16 kernels land).
#include "common.h"

namespace bgw {

int split_workspace_bytes(long long K, int ng, size_t *bytes) {
    (void)K;
    (void)ng;
    *bytes = 0;
    return BGW_OK;
}

int launch_chi_split(const double2 *, long long, int, const double *, int, double, double2 *, int, void *,
                     hipStream_t) {
    set_error("split precision not available in this build");
    return BGW_ERR_UNSUPPORTED;
}

}  // namespace bgw
