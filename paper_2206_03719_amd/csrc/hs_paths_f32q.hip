// hs_paths_f32q.hip -- Greek-set path kernel variants: FP32 paths, Andersen QE (FP64 variance path), FP32 feature storage.
#include "hs_paths.hpp"

namespace hs {

hipError_t launch_paths_f32q(int nmax, int ft, const PathArgs& a, int nchunks, int nbg, hipStream_t st)
{
    if (ft != kFeatF32) return hipErrorInvalidValue;
    return launch_paths_r<float, HS_SCHEME_QE, float>(nmax, a, nchunks, nbg, st);
}

}  // namespace hs
