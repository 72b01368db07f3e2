// BF16 MFMA M2L (placeholder until the matrix-core kernel lands).
#include "plan.h"

namespace fc2t2 {
bool m2l_mfma_supported(const fc2t2_plan_s*) { return false; }
size_t m2l_mfma_table_bytes(const fc2t2_plan_s*) { return 0; }
fc2t2_status m2l_mfma_build_tables(fc2t2_plan_s*, hipStream_t) { return FC2T2_EUNSUPPORTED; }
fc2t2_status launch_m2l_mfma(const fc2t2_plan_s*, int, const void*, void*, bool, bool, hipStream_t) {
  return FC2T2_EUNSUPPORTED;
}
}  // namespace fc2t2
