// search_pq.hip -- batch search and server kernels with compressed (PQ)
// navigation, and the PQ encoder that fills the code rows they read.
//
// The search templates are shared with the full-precision kernels (the
// navigation mode is a template argument of the same kernel); the NAV_PQ
// instances live in one unit per element type (below), so that all of them
// compile in parallel with the full-precision set.
#define FA_SEARCH_TEMPLATES_ONLY
#include "search_kernel.hip"

namespace fa {

// The PQ kernels of each element type are instantiated in a unit of their
// own (search_pq_u8.hip, search_pq_i8.hip, search_pq_f32.hip), so that they
// compile in parallel.
#define FA_PQ_LAUNCHERS(T)                                                                     \
  hipError_t launch_search_pq_##T(const SearchArgs &a, int transport, int wpb, bool pers,      \
                                  hipStream_t st);                                             \
  hipError_t launch_server_pq_##T(const ServerArgs &a, int wpb, int64_t *res, hipStream_t st);
FA_PQ_LAUNCHERS(u8)
FA_PQ_LAUNCHERS(i8)
FA_PQ_LAUNCHERS(f32)
#undef FA_PQ_LAUNCHERS

hipError_t launch_search_pq(const SearchArgs &a, int dtype, int transport, int waves_per_block,
                            bool persistent, hipStream_t st) {
  if (a.pq_m < 1 || a.pq_m > kPqMaxM || !a.pq_codes || !a.pq_cb) return hipErrorInvalidValue;
  switch (dtype) {
    case DT_U8: return launch_search_pq_u8(a, transport, waves_per_block, persistent, st);
    case DT_I8: return launch_search_pq_i8(a, transport, waves_per_block, persistent, st);
    case DT_F32: return launch_search_pq_f32(a, transport, waves_per_block, persistent, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_server_pq(const ServerArgs &a, int dtype, int waves_per_block,
                            int64_t *resident_waves, hipStream_t st) {
  const SearchArgs &b = a.base;
  if (b.pq_m < 1 || b.pq_m > kPqMaxM || !b.pq_codes || !b.pq_cb) return hipErrorInvalidValue;
  switch (dtype) {
    case DT_U8: return launch_server_pq_u8(a, waves_per_block, resident_waves, st);
    case DT_I8: return launch_server_pq_i8(a, waves_per_block, resident_waves, st);
    case DT_F32: return launch_server_pq_f32(a, waves_per_block, resident_waves, st);
    default: return hipErrorInvalidValue;
  }
}

// One block per (128 rows, subspace m): the subspace's 256 centroids and the
// rows' parts in LDS (row stride dsub + 1 floats against bank conflicts);
// thread t finds the nearest centroid of row blockIdx.x * 128 + t.
constexpr int kEncodeRows = 128;
constexpr int kPqMaxDsub = 32;

template <int DT>
__global__ void __launch_bounds__(kEncodeRows) pq_encode_kernel(const uint8_t *nav, int64_t n,
                                                        int nav_stride, int dsub,
                                                        const float *codebooks, uint8_t *codes) {
  extern __shared__ float pq_smem[];
  const int m = blockIdx.y;
  float *cs = pq_smem;                          // 256 x dsub
  float *xs = pq_smem + kPqKsub * dsub;         // kEncodeRows x (dsub + 1)
  const float *cb = codebooks + (int64_t)m * kPqKsub * dsub;
  for (int e = threadIdx.x; e < kPqKsub * dsub; e += blockDim.x) cs[e] = cb[e];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float *x = xs + threadIdx.x * (dsub + 1);
  if (i < n) {
    const uint8_t *row = nav + i * (int64_t)nav_stride;
    for (int j = 0; j < dsub; j++) x[j] = query_elem<DT>(row, m * dsub + j);
  }
  __syncthreads();
  if (i >= n) return;
  float best = 0.0f;
  int bi = 0;
  for (int c = 0; c < kPqKsub; c++) {
    const float *cc = cs + c * dsub;
    float acc = 0.0f;
    for (int j = 0; j < dsub; j++) {
      const float t = x[j] - cc[j];
      acc = fmaf(t, t, acc);
    }
    if (c == 0 || acc < best) {
      best = acc;
      bi = c;
    }
  }
  codes[i * kPqStride + m] = (uint8_t)bi;
}

hipError_t launch_pq_encode(const uint8_t *nav, int64_t n, int nav_stride, int dtype, int d,
                            const float *codebooks, int M, uint8_t *codes, hipStream_t st) {
  if (n < 1 || M < 1 || M > kPqMaxM || d % M != 0 || d / M > kPqMaxDsub)
    return hipErrorInvalidValue;
  const int dsub = d / M;  // LDS: at most 32 KiB of centroids + 16.5 KiB of rows
  const size_t lds = sizeof(float) * ((size_t)kPqKsub * dsub + (size_t)kEncodeRows * (dsub + 1));
  const dim3 grid((unsigned)((n + kEncodeRows - 1) / kEncodeRows), (unsigned)M);
  hipError_t e = hipMemsetAsync(codes, 0, (size_t)n * kPqStride, st);
  if (e != hipSuccess) return e;
  switch (dtype) {
    case DT_U8:
      hipLaunchKernelGGL(pq_encode_kernel<DT_U8>, grid, dim3(kEncodeRows), lds, st, nav, n, nav_stride,
                         dsub, codebooks, codes);
      break;
    case DT_I8:
      hipLaunchKernelGGL(pq_encode_kernel<DT_I8>, grid, dim3(kEncodeRows), lds, st, nav, n, nav_stride,
                         dsub, codebooks, codes);
      break;
    case DT_F32:
      hipLaunchKernelGGL(pq_encode_kernel<DT_F32>, grid, dim3(kEncodeRows), lds, st, nav, n, nav_stride,
                         dsub, codebooks, codes);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fa
