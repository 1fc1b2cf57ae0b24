// Batched persistent kernel, FP32 with leaf size 64.
#include "batched_dev.h"

namespace rtri {
namespace bk {
RTRI_BATCHED_INSTANTIATE(float, 64)
}  // namespace bk
}  // namespace rtri
