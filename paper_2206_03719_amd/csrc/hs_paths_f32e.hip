// hs_paths_f32e.hip -- Greek-set path kernel variants: FP32 paths, full-truncation Euler, FP32 feature storage.
#include "hs_paths.hpp"

namespace hs {

hipError_t launch_paths_f32e(int nmax, int ft, const PathArgs& a, int nchunks, int nbg, hipStream_t st)
{
    if (ft != kFeatF32) return hipErrorInvalidValue;
    return launch_paths_r<float, HS_SCHEME_EULER_FT, float>(nmax, a, nchunks, nbg, st);
}

}  // namespace hs
