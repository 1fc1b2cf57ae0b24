// Batched persistent kernel, FP64 with leaf size 64.
#include "batched_dev.h"

namespace rtri {
namespace bk {
RTRI_BATCHED_INSTANTIATE(double, 64)
}  // namespace bk
}  // namespace rtri
