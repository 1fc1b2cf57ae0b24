// Matrix-core leaf, multiply in F32 (kernel in mleaf_kernel.h).
#include "mleaf_kernel.h"

namespace rtri {

hipError_t mleaf_launch_f32_mult(int nbmax, const LeafDesc &l, hipStream_t st)
{
    return mleaf::launch<float, false>(nbmax, l, st);
}

}  // namespace rtri
