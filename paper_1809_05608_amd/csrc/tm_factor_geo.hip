// Lane kernels of the block-Thomas factor/solve with the geometric flux limiter and the geometric outer
// boundary compiled in (eqs. a23-a26a, a62af): a separate set of instantiations at lower occupancy, launched
// only for problems that ask for either option.
#include "tm_factor_body.hpp"

namespace tmk {

hipError_t launch_factor_geo(const FactorArgs& a, bool fp32, bool transpose, bool pivot, hipStream_t st) {
    return launch_lane<true>(a, fp32, transpose, pivot, st);
}

}  // namespace tmk
