// Two-kernel FP32 query, 64-thread workgroups, wave-shared cells (one instantiation per
// translation unit so that the heavy kernels compile in parallel).
#include "query_split.h"

namespace ksdf {

void launch_query_split_64_wave(const ksdf_model* m, const FastArgs& A, P1Rec* rec, P1Rec* rec2,
                               int* count, int* cursor, int* tsum, void* pws, hipStream_t s) {
  launch_split_nt<64, false>(m, A, rec, rec2, count, cursor, tsum, pws, s);
}

}  // namespace ksdf
