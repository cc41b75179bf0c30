// hs_paths_f64q.hip -- Greek-set path kernel variants: FP64 paths, Andersen QE.
#include "hs_paths.hpp"

namespace hs {

hipError_t launch_paths_f64q(int nmax, int ft, const PathArgs& a, int nchunks, int nbg, hipStream_t st)
{
    if (ft != kFeatF64) return hipErrorInvalidValue;
    return launch_paths_r<double, HS_SCHEME_QE, double>(nmax, a, nchunks, nbg, st);
}

}  // namespace hs
