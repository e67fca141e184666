// Fused exact-search kernels for rows of up to 128 FP32 components.
#include "knn_impl.hpp"

namespace mk {
template mk_status knn_dispatch_k<128>(const float*, int64_t, const float*, const float*, int64_t,
                                       int32_t, int32_t, bool, bool, float*, int64_t*,
                                       hipStream_t, Arena*);
}  // namespace mk
