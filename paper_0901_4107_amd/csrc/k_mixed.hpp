// k_mixed.hpp -- mixed-precision path (placeholder until implemented).
#pragma once

#include "common.hpp"
#include "k_flux.hpp"

namespace mm {

inline int mixed_geo_rows(int D) { return 2 + 2 * D; }

inline mm_status mixed_upload(int, hipStream_t, int64_t, int64_t, const mm_mesh *, const double *, const double *,
                              float *, float *) {
    return MM_E_ARG;
}
inline mm_status mixed_gradients(int, hipStream_t, int64_t, int64_t, double, double, const double *, const double *,
                                 const double *, const double *, const int32_t *, const int32_t *, const int32_t *,
                                 const double *, float *, float *, double *) {
    return MM_E_ARG;
}
inline mm_status mixed_fluxes(int, hipStream_t, int64_t, int64_t, const int32_t *, const int32_t *, const float *,
                              const double *, const double *, const float *, const double *, const float *,
                              const float *, const double *, double, const mm_params &, double *, DiagDev *,
                              int32_t *) {
    return MM_E_ARG;
}

}  // namespace mm
