// Device-side seeded instance generator.  Same counter-based definition as
// the host module (kpgen/__init__.py): SplitMix64's finaliser over
// (seed XOR stream<<56) + (idx+1)*GAMMA, 24 uniform bits per value, values
// u24 * 2^-24 or an inverse-CDF table lookup.  Integer arithmetic only, so the
// bytes equal the host generator's.  Holds no solver arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GAMMA 0x9E3779B97F4A7C15ull

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27; z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}
__device__ __forceinline__ uint32_t u24(uint64_t seed, uint64_t stream, uint64_t idx) {
  const uint64_t base = seed ^ (stream << 56);
  return (uint32_t)(mix64(base + (idx + 1) * GAMMA) >> 40);
}
__device__ __forceinline__ float uval(uint32_t u) { return (float)u * 0x1p-24f; }

__global__ void g_values(uint64_t seed, int stream, uint64_t idx0, int64_t n, const float *table,
                         float *out) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t u = u24(seed, stream, idx0 + t);
    out[t] = table ? table[u] : uval(u);
  }
}

// rows r in [0, nrows): d distinct ascending columns in [0,K), values, rowptr
__global__ void g_csr(uint64_t seed, uint64_t row0, int64_t nrows, int K, int d, int32_t *col,
                      float *val, int64_t *rowptr) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t row = row0 + r;
    int chosen[8];
    for (int t = 0; t < d; ++t) {
      const uint32_t u = u24(seed, 3, row * d + t);
      int k = (int)(((uint64_t)u * (uint64_t)(K - t)) >> 24);
      for (int s = 0; s < t; ++s) k += (k >= chosen[s]);
      int pos = t;
      while (pos > 0 && chosen[pos - 1] > k) { chosen[pos] = chosen[pos - 1]; --pos; }
      chosen[pos] = k;
    }
    for (int t = 0; t < d; ++t) {
      col[r * d + t] = chosen[t];
      val[r * d + t] = uval(u24(seed, 4, row * d + t));
    }
    rowptr[r] = (int64_t)(row0 + r) * d - (int64_t)row0 * d;
    if (r == nrows - 1) rowptr[nrows] = nrows * (int64_t)d;
  }
}

// exact column sums of grid values: sum of round(v * 2^24) per column
__global__ void g_colsum_dense(const float *b, int64_t nrows, int K, unsigned long long *sums) {
  extern __shared__ unsigned long long s[];
  for (int k = threadIdx.x; k < K; k += blockDim.x) s[k] = 0;
  __syncthreads();
  const int64_t n = nrows * K;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long q = (unsigned long long)(b[t] * 0x1p24f);
    atomicAdd(&s[t % K], q);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) atomicAdd(&sums[k], s[k]);
}

__global__ void g_colsum_csr(const int32_t *col, const float *val, int64_t nnz, int K,
                             unsigned long long *sums) {
  extern __shared__ unsigned long long s[];
  for (int k = threadIdx.x; k < K; k += blockDim.x) s[k] = 0;
  __syncthreads();
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nnz;
       t += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long q = (unsigned long long)(val[t] * 0x1p24f);
    atomicAdd(&s[col[t]], q);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) atomicAdd(&sums[k], s[k]);
}

static int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b > 16384 ? 16384 : (b < 1 ? 1 : b));
}

extern "C" {
int kpgen_values(uint64_t seed, int stream, uint64_t idx0, int64_t n, const float *table,
                 float *out, void *hstream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(g_values, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hstream, seed, stream,
                     idx0, n, table, out);
  return (int)hipGetLastError();
}
int kpgen_csr(uint64_t seed, uint64_t row0, int64_t nrows, int K, int d, int32_t *col, float *val,
              int64_t *rowptr, void *hstream) {
  if (nrows <= 0 || d < 1 || d > 8 || d > K) return -1;
  hipLaunchKernelGGL(g_csr, dim3(grid_for(nrows)), dim3(256), 0, (hipStream_t)hstream, seed, row0,
                     nrows, K, d, col, val, rowptr);
  return (int)hipGetLastError();
}
int kpgen_colsum_dense(const float *b, int64_t nrows, int K, unsigned long long *sums,
                       void *hstream) {
  if (nrows <= 0) return 0;
  hipLaunchKernelGGL(g_colsum_dense, dim3(grid_for(nrows * K)), dim3(256), K * 8,
                     (hipStream_t)hstream, b, nrows, K, sums);
  return (int)hipGetLastError();
}
int kpgen_colsum_csr(const int32_t *col, const float *val, int64_t nnz, int K,
                     unsigned long long *sums, void *hstream) {
  if (nnz <= 0) return 0;
  hipLaunchKernelGGL(g_colsum_csr, dim3(grid_for(nnz)), dim3(256), K * 8, (hipStream_t)hstream,
                     col, val, nnz, K, sums);
  return (int)hipGetLastError();
}
}
