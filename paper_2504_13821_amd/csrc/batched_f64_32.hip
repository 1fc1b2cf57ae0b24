// Batched persistent kernel, FP64 with leaf size 32.
#include "batched_dev.h"

namespace rtri {
namespace bk {
RTRI_BATCHED_INSTANTIATE(double, 32)
}  // namespace bk
}  // namespace rtri
