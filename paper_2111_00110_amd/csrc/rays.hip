// Ray layers (placeholder).
#include "plan.h"

namespace fc2t2 {
size_t ray_integral_bwd_ws(const fc2t2_plan_s*, int64_t) { return 0; }
fc2t2_status launch_ray_integral(const fc2t2_plan_s*, const void*, const void*, const void*, double,
                                 double, int64_t, void*, hipStream_t) { return FC2T2_EUNSUPPORTED; }
fc2t2_status ray_integral_backward(const fc2t2_plan_s*, const void*, const void*, double, double,
                                   int64_t, const void*, void*, void*, hipStream_t) { return FC2T2_EUNSUPPORTED; }
fc2t2_status launch_ray_root(const fc2t2_plan_s*, const void*, const void*, const void*, double, double,
                             int64_t, double, void*, void*, int32_t*, void*, hipStream_t) { return FC2T2_EUNSUPPORTED; }
size_t ray_root_bwd_ws(const fc2t2_plan_s*, int64_t) { return 0; }
fc2t2_status ray_root_backward(const fc2t2_plan_s*, const void*, const int32_t*, int64_t, const void*,
                               const void*, void*, void*, hipStream_t) { return FC2T2_EUNSUPPORTED; }
}  // namespace fc2t2

extern "C" {
fc2t2_status fc2t2_ray_integral(fc2t2_plan, const void*, const void*, const void*, double, double,
                                int64_t, void*, hipStream_t) { return FC2T2_EUNSUPPORTED; }
fc2t2_status fc2t2_ray_integral_backward(fc2t2_plan, const void*, const void*, double, double, int64_t,
                                         const void*, void*, void*, size_t, hipStream_t) { return FC2T2_EUNSUPPORTED; }
fc2t2_status fc2t2_ray_root(fc2t2_plan, const void*, const void*, const void*, double, double, int64_t,
                            double, void*, void*, int32_t*, void*, hipStream_t) { return FC2T2_EUNSUPPORTED; }
fc2t2_status fc2t2_ray_root_backward(fc2t2_plan, const void*, const int32_t*, int64_t, const void*,
                                     const void*, void*, void*, size_t, hipStream_t) { return FC2T2_EUNSUPPORTED; }
}
