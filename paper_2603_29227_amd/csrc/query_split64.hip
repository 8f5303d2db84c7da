// Two-kernel FP32 query, 64-thread workgroups.
#include "query_split.h"

namespace ksdf {

void launch_query_split_64(const ksdf_model* m, const FastArgs& A, Pass1* rec, Pass1* rec2,
                            int* count, int* cursor, int* tsum, bool lane, void* pws,
                            hipStream_t s) {
  if (lane) launch_split_nt<64, true>(m, A, rec, rec2, count, cursor, tsum, pws, s);
  else launch_split_nt<64, false>(m, A, rec, rec2, count, cursor, tsum, pws, s);
}

}  // namespace ksdf
