// Two-kernel FP32 query, 256-thread workgroups, per-lane cells (one instantiation per
// translation unit so that the heavy kernels compile in parallel).
#include "query_split.h"

namespace ksdf {

void launch_query_split_256_lane(const ksdf_model* m, const FastArgs& A, P1Rec* rec, P1Rec* rec2,
                               int* count, int* cursor, int* tsum, void* pws, hipStream_t s) {
  launch_split_nt<256, true>(m, A, rec, rec2, count, cursor, tsum, pws, s);
}

}  // namespace ksdf
