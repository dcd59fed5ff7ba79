// Lane kernels of the block-Thomas factor/solve (bodies in tm_factor_body.hpp): the instantiations without
// the geometric options, and the dispatch of every factor launch (the quad kernel, these, or the geometric
// instantiations of tm_factor_geo.hip).
#include "tm_factor_body.hpp"

namespace tmk {

size_t factor_ws_bytes_per_system(int I, int N, bool fp32) {
    const int NT = padded_groups(N);
    if (NT < 0) return 0;
    const size_t es = fp32 ? 4 : 8;
    return (size_t)I * NT * (NT + 1) * es;
}

hipError_t launch_factor(const FactorArgs& a, bool fp32, bool transpose, bool pivot, hipStream_t st, int kernel) {
    // the float32 forward solve with diagonal pivots (the mixed-precision Newton update) takes one
    // system per quad of lanes up to 20 groups
    if (kernel != kFactorLane && fp32 && !transpose && !pivot &&
        launch_factor_quad(a, st, kernel))
        return hipGetLastError();
    if (a.sh.limiter == 2 || a.sh.outer_bc == 2) return launch_factor_geo(a, fp32, transpose, pivot, st);
    return launch_lane<false>(a, fp32, transpose, pivot, st);
}

}  // namespace tmk
