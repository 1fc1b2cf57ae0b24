// Matrix-core leaf, multiply in F64 (kernel in mleaf_kernel.h).
#include "mleaf_kernel.h"

namespace rtri {

hipError_t mleaf_launch_f64_mult(int nbmax, const LeafDesc &l, hipStream_t st)
{
    return mleaf::launch<double, false>(nbmax, l, st);
}

}  // namespace rtri
