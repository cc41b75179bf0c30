// hs_paths_f32h.hip -- Greek-set path kernel variants: FP32 paths, full-truncation Euler, FP16 or BF16 feature storage.
#include "hs_paths.hpp"

namespace hs {

hipError_t launch_paths_f32h(int nmax, int ft, const PathArgs& a, int nchunks, int nbg, hipStream_t st)
{
    switch (ft) {
    case kFeatF16: return launch_paths_r<float, HS_SCHEME_EULER_FT, _Float16>(nmax, a, nchunks, nbg, st);
    case kFeatBF16: return launch_paths_r<float, HS_SCHEME_EULER_FT, __bf16>(nmax, a, nchunks, nbg, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hs
