// Internal declarations of the multicoil MRI kernels (k_mri.hip) used by the
// C ABI in capi_mri.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "skei_internal.h"
#include "skei_mri.h"

namespace skei {

constexpr int kMriMaxN = SKEI_MRI_MAX_N;

bool mri_size_ok(int n);   // a power of two in [4, kMriMaxN]
int launch_mri_fwd(const float2 *maps, int nc, int n, const float2 *x, int batch, const float *mask,
                   const float *wgt, float2 *k, hipStream_t st);
int launch_mri_adj(const float2 *maps, int nc, int n, const float2 *k, int batch, const float *mask,
                   const float *wgt, float2 *x, float2 *work, hipStream_t st);
int launch_coil_mix(const float2 *G, int m_out, int l_in, const float2 *z, long long d, int batch, float2 *out,
                    hipStream_t st);
int launch_coil_weights(const float2 *maps, int nc, long long d, float *wgt, hipStream_t st);
int launch_coil_cov(const float2 *k, int nc, long long d, double *V, hipStream_t st);

}  // namespace skei
