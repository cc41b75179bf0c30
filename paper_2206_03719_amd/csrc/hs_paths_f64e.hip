// hs_paths_f64e.hip -- Greek-set path kernel variants: FP64 paths, full-truncation Euler.
#include "hs_paths.hpp"

namespace hs {

hipError_t launch_paths_f64e(int nmax, int ft, const PathArgs& a, int nchunks, int nbg, hipStream_t st)
{
    if (ft != kFeatF64) return hipErrorInvalidValue;
    return launch_paths_r<double, HS_SCHEME_EULER_FT, double>(nmax, a, nchunks, nbg, st);
}

}  // namespace hs
