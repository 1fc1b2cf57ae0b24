// Batched persistent kernel, FP32 with leaf size 32.
#include "batched_dev.h"

namespace rtri {
namespace bk {
RTRI_BATCHED_INSTANTIATE(float, 32)
}  // namespace bk
}  // namespace rtri
