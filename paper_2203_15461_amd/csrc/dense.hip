// Dense FP64 linear algebra on CDNA4 matrix cores and the HBM-streaming solve.
//
// The paper obtains the capacitance matrix by inverting the elastance A
// (Sec. II.A, Eq. 3) and projects it onto the charge-neutral subspace (Eq. 4).
// Here A = L L^T by a blocked right-looking Cholesky (64-wide panels: a
// one-workgroup diagonal factorisation, a panel solve and a trailing
// symmetric update as MFMA GEMMs), X = L^-1 by blocked forward substitution,
// and A^-1 = X^T X as a triangular-aware MFMA GEMM.
//
// v_mfma_f64_16x16x4f64 operand layout (lane l of a wave64):
//   A operand: element (row l%16, k l/16); B operand: (k l/16, col l%16);
//   result register r: element (row l/16 + 4 r, col l%16).
#include <algorithm>
#include <cstdlib>

#include "cpm_internal.h"

namespace cpm {

typedef double v4d __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// GEMM: C = beta C + alpha op(A) op(B), 64x64 tile per 256-thread workgroup,
// each wave a 32x32 quadrant of 2x2 MFMA blocks, K staged through LDS in
// slabs of 16 with the next slab prefetched into registers.
// ---------------------------------------------------------------------------
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm_f64(int M, int N, int K, double alpha,
                                                  const double* __restrict__ A, int lda,
                                                  const double* __restrict__ B, int ldb,
                                                  double beta, double* C, int ldc, int tri,
                                                  int kmode, const int* __restrict__ rowmap) {
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  if (tri && n0 > m0) return;
  const int kbeg = kmode ? (m0 > n0 ? m0 : n0) : 0;
  __shared__ double As[16][64 + 4];
  __shared__ double Bs[16][64 + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  v4d acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};

  double ra[4], rb[4];
  auto load = [&](int k0) {
    if (!TA) {
      const int r = tid >> 2, c = (tid & 3) * 4;
      const double* src = A + (size_t)(m0 + r) * lda + k0 + c;
      for (int t = 0; t < 4; ++t) ra[t] = src[t];
    } else {
      const int r = tid >> 4, c = (tid & 15) * 4;
      const double* src = A + (size_t)(k0 + r) * lda + m0 + c;
      for (int t = 0; t < 4; ++t) ra[t] = src[t];
    }
    if (!TB) {
      const int r = tid >> 4, c = (tid & 15) * 4;
      const double* src = B + (size_t)(k0 + r) * ldb + n0 + c;
      for (int t = 0; t < 4; ++t) rb[t] = src[t];
    } else {
      const int r = tid >> 2, c = (tid & 3) * 4;
      const double* src = B + (size_t)(n0 + r) * ldb + k0 + c;
      for (int t = 0; t < 4; ++t) rb[t] = src[t];
    }
  };
  auto store = [&]() {
    if (!TA) {
      const int r = tid >> 2, c = (tid & 3) * 4;
      for (int t = 0; t < 4; ++t) As[c + t][r] = ra[t];
    } else {
      const int r = tid >> 4, c = (tid & 15) * 4;
      for (int t = 0; t < 4; ++t) As[r][c + t] = ra[t];
    }
    if (!TB) {
      const int r = tid >> 4, c = (tid & 15) * 4;
      for (int t = 0; t < 4; ++t) Bs[r][c + t] = rb[t];
    } else {
      const int r = tid >> 2, c = (tid & 3) * 4;
      for (int t = 0; t < 4; ++t) Bs[c + t][r] = rb[t];
    }
  };

  if (kbeg < K) load(kbeg);
  for (int k0 = kbeg; k0 < K; k0 += 16) {
    store();
    __syncthreads();
    if (k0 + 16 < K) load(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int kr = kk + (lane >> 4), cc = lane & 15;
      const double a0 = As[kr][wm + cc], a1 = As[kr][wm + 16 + cc];
      const double b0 = Bs[kr][wn + cc], b1 = Bs[kr][wn + 16 + cc];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        int row = m0 + wm + a * 16 + (lane >> 4) + 4 * r;
        if (rowmap) {                                  // scattered output rows (-1: skip)
          row = rowmap[row];
          if (row < 0) continue;
        }
        const int col = n0 + wn + b * 16 + (lane & 15);
        double* cp = C + (size_t)row * ldc + col;
        const double v = alpha * acc[a][b][r];
        *cp = (beta != 0.0) ? v + beta * (*cp) : v;
      }
}

void launch_gemm_f64(hipStream_t st, bool transA, bool transB, int M, int N, int K, double alpha,
                     const double* A, int lda, const double* B, int ldb, double beta, double* C,
                     int ldc, int tri, int kmode, const int* rowmap) {
  if (M <= 0 || N <= 0) return;
  dim3 grid(N / 64, M / 64), block(256);
  if (!transA && !transB)
    hipLaunchKernelGGL((k_gemm_f64<false, false>), grid, block, 0, st, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, tri, kmode, rowmap);
  else if (!transA && transB)
    hipLaunchKernelGGL((k_gemm_f64<false, true>), grid, block, 0, st, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, tri, kmode, rowmap);
  else if (transA && !transB)
    hipLaunchKernelGGL((k_gemm_f64<true, false>), grid, block, 0, st, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, tri, kmode, rowmap);
  else
    hipLaunchKernelGGL((k_gemm_f64<true, true>), grid, block, 0, st, M, N, K, alpha, A, lda, B,
                       ldb, beta, C, ldc, tri, kmode, rowmap);
}

// ---------------------------------------------------------------------------
// Diagonal 64x64 block of the Cholesky factorisation, in one workgroup, in
// four panels of 16 columns: wave 0 factors the panel's 16 x 16 diagonal
// block right-looking in registers (cross-lane moves), one thread per row below
// solves that row's 16 panel entries, then every thread updates trailing
// elements.  The inverse of the factor: the four diagonal 16 x 16 blocks by
// forward substitution (a wave each, a lane per column), then block rows 1..3
// in turn, X_ik = -X_ii sum_{j=k}^{i-1} L_ij X_jk.  About 20 workgroup
// barriers in all.  A pivot <= 0 (or NaN) records 1 + its global index in
// *flag (first one wins) and continues with 1.
// ---------------------------------------------------------------------------
// lane l's value of v, in every lane (l uniform)
__device__ inline double readlane_f64(double v, int l) {
  const unsigned long long x = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__global__ void __launch_bounds__(1024) k_potrf_diag(double* Lblk, int ld, double* Dinv, int* flag,
                                                     int k0) {
  __shared__ double a[64][65];     // working lower triangle, becomes L
  __shared__ double X[64][65];     // L^-1
  __shared__ double T[3][16][17];  // block-row products of the inverse
  __shared__ double rd[64];        // 1 / L[j][j]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  {
    // four entries per thread, their loads all in flight at once
    double t[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 1024 * u, r = e >> 6, c = e & 63;
      t[u] = (c <= r) ? Lblk[(size_t)r * ld + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 1024 * u, r = e >> 6, c = e & 63;
      a[r][c] = t[u];
      X[r][c] = 0.0;
    }
  }
  __syncthreads();
  for (int p0 = 0; p0 < 64; p0 += 16) {
    if (wave == 0) {
      // lane (r, part) keeps row p0 + r, columns p0 + 4 part .. + 3, of the
      // panel's diagonal block in registers; step j reads the pivot and the
      // entries of column j from the lanes that own them (cross-lane moves),
      // so no step waits on LDS
      const int r = lane & 15, part = lane >> 4;
      double v[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) v[s] = a[p0 + r][p0 + 4 * part + s];
      double rdl = 0.0;                    // 1 / L[p0 + r][p0 + r]
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int pj = j >> 2, sj = j & 3;   // owner part and slot of column j
        double piv = readlane_f64(v[sj], j + 16 * pj);
        if (!(piv > 0.0)) {
          if (lane == 0) atomicCAS(flag, 0, k0 + p0 + j + 1);
          piv = 1.0;
        }
        const double d = sqrt(piv), rdj = 1.0 / d;
        const double arj = __shfl(v[sj], r + 16 * pj, 64);       // L[r][j] before scaling
        double acj[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) acj[s] = __shfl(v[sj], 4 * part + s + 16 * pj, 64);
        const double lr = arj * rdj;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int c = 4 * part + s;
          if (c > j && c <= r) v[s] -= lr * (acj[s] * rdj);
        }
        if (part == pj) {
          if (r > j) v[sj] = lr;
          else if (r == j) v[sj] = d;
        }
        if (r == j) rdl = rdj;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (4 * part + s <= r) a[p0 + r][p0 + 4 * part + s] = v[s];
      if (part == 0) rd[p0 + r] = rdl;
    }
    __syncthreads();
    const int nrem = 64 - p0 - 16;
    if (tid < nrem) {                      // row R of the panel below the diagonal block
      const int R = p0 + 16 + tid;
      double row[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) row[t] = a[R][p0 + t];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        double s = row[j];
#pragma unroll
        for (int t = 0; t < j; ++t) s -= row[t] * a[p0 + j][p0 + t];
        row[j] = s * rd[p0 + j];
      }
#pragma unroll
      for (int t = 0; t < 16; ++t) a[R][p0 + t] = row[t];
    }
    __syncthreads();
    for (int e = tid; e < nrem * nrem; e += 1024) {
      const int R = p0 + 16 + e / nrem, C = p0 + 16 + e % nrem;
      if (C <= R) {
        double s = a[R][C];
#pragma unroll
        for (int t = 0; t < 16; ++t) s -= a[R][p0 + t] * a[C][p0 + t];
        a[R][C] = s;
      }
    }
    __syncthreads();
  }
  // diagonal blocks of X: wave k inverts L_kk, lane c solves column c
  if (wave < 4 && lane < 16) {
    // entries above the diagonal of the column stay zero: x[t] = 0 for t < c
    const int p0 = 16 * wave, c = lane;
    double x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      double s = (r == c) ? 1.0 : 0.0;
#pragma unroll
      for (int t = 0; t < r; ++t) s -= a[p0 + r][p0 + t] * x[t];
      x[r] = (r >= c) ? s * rd[p0 + r] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) X[p0 + r][p0 + c] = x[r];
  }
  __syncthreads();
  for (int i = 1; i < 4; ++i) {
    const int k = tid >> 8, r = (tid >> 4) & 15, c = tid & 15;
    if (k < i) {
      double s = 0.0;
      for (int j = k; j < i; ++j)
#pragma unroll
        for (int t = 0; t < 16; ++t) s += a[16 * i + r][16 * j + t] * X[16 * j + t][16 * k + c];
      T[k][r][c] = s;
    }
    __syncthreads();
    if (k < i) {
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < 16; ++t) s += X[16 * i + r][16 * i + t] * T[k][t][c];
      X[16 * i + r][16 * k + c] = -s;
    }
    __syncthreads();
  }
  for (int e = tid; e < 64 * 64; e += 1024) {
    const int r = e >> 6, c = e & 63;
    Lblk[(size_t)r * ld + c] = (c <= r) ? a[r][c] : 0.0;
    Dinv[e] = X[r][c];
  }
}

void launch_potrf_diag(hipStream_t st, double* Lblk, int ld, double* Dinv, int* flag, int k0) {
  hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(1024), 0, st, Lblk, ld, Dinv, flag, k0);
}

__global__ void k_set_identity(int npad, double* X) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)npad * npad) return;
  const int i = (int)(e / npad), j = (int)(e % npad);
  X[e] = (i == j) ? 1.0 : 0.0;
}

void launch_set_identity(hipStream_t st, int npad, double* X) {
  const size_t tot = (size_t)npad * npad;
  hipLaunchKernelGGL(k_set_identity, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, npad,
                     X);
}

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum of 256 threads in a fixed order; result valid in every thread
__device__ inline double block_sum256(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return t;
}

// sum over a 1024-thread workgroup: wave sums, then the 16 in wave order
__device__ inline double block_sum1024(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < 16; ++w) t += sh[w];
  __syncthreads();
  return t;
}

// out[i] = sum_{j<n} M[i][j] for i < n (one wave per row, fixed order)
__global__ void k_row_sums(int n, int npad, const double* __restrict__ M, double* out) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n) return;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += M[(size_t)row * npad + j];
  s = wave_sum(s);
  if (lane == 0) out[row] = s;
}

void launch_row_sums(hipStream_t st, int n, int npad, const double* M, double* out) {
  hipLaunchKernelGGL(k_row_sums, dim3((n + 3) / 4), dim3(256), 0, st, n, npad, M, out);
}

__global__ void k_sum_vector(int n, const double* __restrict__ v, double* out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += v[i];
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) *out = s;
}

void launch_sum_vector(hipStream_t st, int n, const double* v, double* out) {
  hipLaunchKernelGGL(k_sum_vector, dim3(1), dim3(256), 0, st, n, v, out);
}

// S = A^-1 - u u^T / s on the n x n block (Eq. 4); zero in the padding.
__global__ void k_make_S(int n, int npad, const double* __restrict__ Ainv,
                         const double* __restrict__ u, const double* __restrict__ s_dev,
                         double* __restrict__ S) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)npad * npad) return;
  const int i = (int)(e / npad), j = (int)(e % npad);
  double v = 0.0;
  if (i < n && j < n) v = Ainv[e] - u[i] * u[j] / (*s_dev);
  S[e] = v;
}

void launch_make_S(hipStream_t st, int n, int npad, const double* Ainv, const double* u,
                   const double* s_dev, double* S) {
  const size_t tot = (size_t)npad * npad;
  hipLaunchKernelGGL(k_make_S, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, npad,
                     Ainv, u, s_dev, S);
}

// round-to-nearest-even FP32 -> BF16
__device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t x = __float_as_uint(f);
  if ((x & 0x7f800000u) == 0x7f800000u) return (uint16_t)(x >> 16);
  x += 0x7fffu + ((x >> 16) & 1u);
  return (uint16_t)(x >> 16);
}

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// FP32 copy and split-BF16 pair of S (hi = bf16(S), lo = bf16(S - hi)).
__global__ void k_convert_S(size_t tot, const double* __restrict__ S, float* S32, uint16_t* hi,
                            uint16_t* lo) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= tot) return;
  const double v = S[e];
  if (S32) S32[e] = (float)v;
  if (hi) {
    const uint16_t h = f32_to_bf16((float)v);
    hi[e] = h;
    lo[e] = f32_to_bf16((float)(v - (double)bf16_to_f32(h)));
  }
}

// x ~ hi + lo: hi = bf16(x), lo = bf16(x - hi) through FP32, as for S
__global__ void k_split_bf16(size_t count, const double* __restrict__ x, uint16_t* __restrict__ hi,
                             uint16_t* __restrict__ lo) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const float f = (float)x[e];
  const uint16_t h = f32_to_bf16(f);
  hi[e] = h;
  lo[e] = f32_to_bf16(f - bf16_to_f32(h));
}

void launch_split_bf16(hipStream_t st, size_t count, const double* x, uint16_t* hi, uint16_t* lo) {
  hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count,
                     x, hi, lo);
}

void launch_convert_S(hipStream_t st, int npad, const double* S, float* S32, uint16_t* hi,
                      uint16_t* lo) {
  const size_t tot = (size_t)npad * npad;
  hipLaunchKernelGGL(k_convert_S, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, tot, S,
                     S32, hi, lo);
}

// ---------------------------------------------------------------------------
// Matrix-vector product y[b] = sign * M x[b] + addscale * add, streaming the
// npad x npad matrix M (FP64 or FP32) once per vector.  x is FP64, npad
// apart per vector and zero beyond n, so every load is an aligned 16-byte
// vector with no bounds test.  One wave per R consecutive rows: 16-byte
// coalesced loads of each row, every x element read once per wave (through
// the cache) for all R rows, FP64 accumulation, wave reductions in a fixed
// order.  Matrices larger than the last-level cache are read with
// nontemporal loads (streamed past the caches, which the x vector keeps).
// ---------------------------------------------------------------------------
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename TM, int R, bool NT>
__global__ void __launch_bounds__(256) k_matvec(int npad, const TM* __restrict__ M,
                                                const double* __restrict__ x,
                                                const double* __restrict__ add, int add_ld,
                                                double addscale, double* __restrict__ y, int ldy,
                                                int negate) {
  const int lane = threadIdx.x & 63;
  const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * R;   // R consecutive rows per wave
  const int b = blockIdx.y;
  if (row0 >= npad) return;                  // npad is a multiple of 64, so all R rows exist
  constexpr int VEC = 16 / sizeof(TM);
  const TM* mrow = M + (size_t)row0 * npad;
  const double* xb = x + (size_t)b * npad;
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
#pragma unroll 2
  for (int j0 = lane * VEC; j0 < npad; j0 += 64 * VEC) {
    // the R row segments first (R x 16 B in flight per lane), then x once for all rows
    TM mv[R][VEC];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const TM* src = mrow + (size_t)r * npad + j0;
      if constexpr (VEC == 2) {
        const d2v t = NT ? __builtin_nontemporal_load(reinterpret_cast<const d2v*>(src))
                         : *reinterpret_cast<const d2v*>(src);
        mv[r][0] = t.x; mv[r][1] = t.y;
      } else {
        const f4v t = NT ? __builtin_nontemporal_load(reinterpret_cast<const f4v*>(src))
                         : *reinterpret_cast<const f4v*>(src);
        mv[r][0] = t.x; mv[r][1] = t.y; mv[r][2] = t.z; mv[r][3] = t.w;
      }
    }
    double xj[VEC];
#pragma unroll
    for (int t = 0; t < VEC; t += 2) {
      const d2v v = *reinterpret_cast<const d2v*>(xb + j0 + t);
      xj[t] = v.x; xj[t + 1] = v.y;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int t = 0; t < VEC; ++t) acc[r] += (double)mv[r][t] * xj[t];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = wave_sum(acc[r]);
  if (lane < R) {
    double s = acc[0];
#pragma unroll
    for (int r = 1; r < R; ++r)
      if (lane == r) s = acc[r];
    const int row = row0 + lane;
    double v = negate ? -s : s;
    if (add) v += addscale * add[(size_t)b * add_ld + row];
    y[(size_t)b * ldy + row] = v;
  }
}

template <typename TM>
void launch_matvec_t(hipStream_t st, int npad, const TM* M, int batch, const double* x,
                     const double* add, int add_ld, double addscale, double* y, int ldy,
                     int negate) {
  // rows per wave: 4 rows share each x load from npad = 2048 on (measured
  // best both where S stays in the last-level cache, n ~ 3k, and where it
  // streams from HBM, n ~ 20k); nontemporal loads from 128 MiB of matrix on
  // (20096^2: FP32 84%, FP64 87% of the HBM peak against 75%, 78% with
  // ordinary loads; a matrix that fits the 256 MB cache loses by them)
  int R = npad >= 2048 ? 4 : npad >= 1024 ? 2 : 1;
  bool nt = (double)npad * npad * sizeof(TM) >= 128.0 * 1024 * 1024;
  if (const char* ev = std::getenv("CPM_MV_ROWS")) {
    const int r = std::atoi(ev);
    if (r == 1 || r == 2 || r == 4 || r == 8) R = r;
  }
  if (const char* ev = std::getenv("CPM_MV_NT")) nt = std::atoi(ev) != 0;
  dim3 grid((npad / R + 3) / 4, batch), block(256);
#define CPM_MV(RR, NN)                                                                     \
  hipLaunchKernelGGL((k_matvec<TM, RR, NN>), grid, block, 0, st, npad, M, x, add, add_ld,  \
                     addscale, y, ldy, negate)
  if (nt) {
    if (R == 8) CPM_MV(8, true); else if (R == 4) CPM_MV(4, true);
    else if (R == 2) CPM_MV(2, true); else CPM_MV(1, true);
  } else {
    if (R == 8) CPM_MV(8, false); else if (R == 4) CPM_MV(4, false);
    else if (R == 2) CPM_MV(2, false); else CPM_MV(1, false);
  }
#undef CPM_MV
}

// One matrix-vector product per right-hand side: y = M x (+ add), M npad x
// npad row-major (FP64 or FP32), x FP64 padded (npad apart, zero beyond n),
// streamed once per vector with 16-byte coalesced loads; R rows per wave
// share each x load; fixed-order wave reductions.
void launch_matvec(hipStream_t st, int which, int npad, const void* M, int batch, const double* x,
                   const double* add, int add_ld, double addscale, double* y, int ldy, int negate) {
  if (which == 0)
    launch_matvec_t(st, npad, (const double*)M, batch, x, add, add_ld, addscale, y, ldy, negate);
  else
    launch_matvec_t(st, npad, (const float*)M, batch, x, add, add_ld, addscale, y, ldy, negate);
}

// dst[b] (npad apart, FP64) = src[b] (ldx apart, FP64 or FP32) minus its mean
// over i < n when `center` (the same fixed-order sum as k_row_means), zero
// for n <= i < npad: the padded right-hand side of the streaming solve.
// Grid (batch, parts): every workgroup of a vector forms the same mean (the
// same order; four loads per thread in flight) and writes its own part, so a
// single vector is not left to one workgroup.
template <typename TX>
__global__ void __launch_bounds__(1024) k_center_pad(int n, int npad, const TX* __restrict__ x,
                                                     int ldx, int center,
                                                     double* __restrict__ dst) {
  __shared__ double sh[16];
  const TX* xb = x + (size_t)blockIdx.x * ldx;
  double mean = 0.0;
  if (center) {
    double s = 0.0;
    for (int i0 = threadIdx.x; i0 < n; i0 += 4096) {
      double v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = (double)xb[min(i0 + 1024 * j, n - 1)];
#pragma unroll
      for (int j = 0; j < 4; ++j) s += i0 + 1024 * j < n ? v[j] : 0.0;
    }
    mean = block_sum1024(s, sh) / n;
  }
  double* out = dst + (size_t)blockIdx.x * npad;
  for (int i = blockIdx.y * 1024 + threadIdx.x; i < npad; i += 1024 * gridDim.y)
    out[i] = i < n ? (double)xb[i] - mean : 0.0;
}

// workgroups per vector of the two per-vector passes: all of the vector's
// 1024-element parts for small batches, one otherwise
static int vector_parts(int batch, int len) {
  return batch < 16 ? std::max(1, (len + 1023) / 1024) : 1;
}

void launch_center_pad(hipStream_t st, int n, int npad, int batch, const void* x, int x_is_f32,
                       int ldx, int center, double* dst) {
  const dim3 grid(batch, vector_parts(batch, npad));
  if (x_is_f32)
    hipLaunchKernelGGL(k_center_pad<float>, grid, dim3(1024), 0, st, n, npad,
                       static_cast<const float*>(x), ldx, center, dst);
  else
    hipLaunchKernelGGL(k_center_pad<double>, grid, dim3(1024), 0, st, n, npad,
                       static_cast<const double*>(x), ldx, center, dst);
}

// means[b] = (1/n) sum_{i<n} x[b][i]: the uniform part of a right-hand side.
// S e = 0, so S x = S (x - mean e); removing it first keeps the rounding of a
// low-precision S from acting on the (large) uniform potential.
__global__ void __launch_bounds__(1024) k_row_means(int n, const void* __restrict__ x, int x_is_f32,
                                                    int ldx, double* __restrict__ means) {
  __shared__ double sh[16];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024)
    s += x_is_f32 ? (double)reinterpret_cast<const float*>(x)[(size_t)b * ldx + i]
                  : reinterpret_cast<const double*>(x)[(size_t)b * ldx + i];
  s = block_sum1024(s, sh);
  if (threadIdx.x == 0) means[b] = s / n;
}

void launch_row_means(hipStream_t st, int n, int batch, const void* x, int x_is_f32, int ldx,
                      double* means) {
  hipLaunchKernelGGL(k_row_means, dim3(batch), dim3(1024), 0, st, n, x, x_is_f32, ldx, means);
}

// x[b][i] -= mean_b over i < n (in place, FP64, stride ld)
__global__ void __launch_bounds__(1024) k_center_rows(int n, int ld, double* __restrict__ x) {
  __shared__ double sh[16];
  double* row = x + (size_t)blockIdx.x * ld;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) s += row[i];
  s = block_sum1024(s, sh) / n;
  for (int i = threadIdx.x; i < n; i += 1024) row[i] -= s;
}

void launch_center_rows(hipStream_t st, int n, int ld, int batch, double* x) {
  hipLaunchKernelGGL(k_center_rows, dim3(batch), dim3(1024), 0, st, n, ld, x);
}

// c[b] = b[b] + v (FP64, npad stride, zero padding): the right-hand side of
// A q = b + v used by the refinement residual.
__global__ void k_make_rhs(int n, int npad, const void* __restrict__ bsrc, int b_is_f32,
                           const double* __restrict__ v, double* __restrict__ c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
  if (i >= npad) return;
  double x = 0.0;
  if (i < n)
    x = (b_is_f32 ? (double)reinterpret_cast<const float*>(bsrc)[(size_t)b * n + i]
                  : reinterpret_cast<const double*>(bsrc)[(size_t)b * n + i]) + v[i];
  c[(size_t)b * npad + i] = x;
}

void launch_make_rhs(hipStream_t st, int n, int npad, int batch, const void* bsrc, int b_is_f32,
                     const double* v, double* c) {
  hipLaunchKernelGGL(k_make_rhs, dim3((npad + 255) / 256, batch), dim3(256), 0, st, n, npad, bsrc,
                     b_is_f32, v, c);
}

// ---------------------------------------------------------------------------
// Neutrality projection and electrode totals (FP64):
//   mu = e^T qt / s,  q = qt - mu u,  Q_alpha = T_alpha - mu U_alpha,
// with T_alpha and U_alpha the sums of qt and u over electrode alpha (equal
// to the sum of q over alpha).  Grid (batch, parts): every workgroup of a
// vector forms the same e^T qt (one fixed-order workgroup sum) and writes its
// own part of q; workgroup 0 also forms the electrode sums, four electrodes
// per pass, the first four in the pass that sums e^T qt.
// ---------------------------------------------------------------------------
template <bool ADD>
__global__ void __launch_bounds__(1024) k_finalize(int n, const double* __restrict__ qt, int ldqt,
                                                   const double* __restrict__ add,
                                                   const double* __restrict__ u,
                                                   const double* __restrict__ s_dev,
                                                   const int* __restrict__ eid, int n_e,
                                                   double* __restrict__ q, int ldq,
                                                   double* __restrict__ Qe) {
  __shared__ double sh[16];
  __shared__ double shq[8][16];
  const int b = blockIdx.x;
  const double* x = qt + (size_t)b * ldqt;
  auto val = [&](int i) { return ADD ? x[i] + add[i] : x[i]; };
  const bool totals = Qe && blockIdx.y == 0;
  double s = 0.0, t[4] = {0.0, 0.0, 0.0, 0.0}, w[4] = {0.0, 0.0, 0.0, 0.0};
  // four elements per thread in flight: i0 + 1024 j, in increasing order
  for (int i0 = threadIdx.x; i0 < n; i0 += 4096) {
    double v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = val(min(i0 + 1024 * j, n - 1));
    if (totals) {
      double uu[4];
      int e[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = min(i0 + 1024 * j, n - 1);
        uu[j] = u[i];
        e[j] = i0 + 1024 * j < n ? eid[i] : -1;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          t[k] += e[j] == k ? v[j] : 0.0;
          w[k] += e[j] == k ? uu[j] : 0.0;
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) s += i0 + 1024 * j < n ? v[j] : 0.0;
  }
  s = block_sum1024(s, sh);
  const double mu = s / (*s_dev);
  double* qo = q + (size_t)b * ldq;
  for (int i = blockIdx.y * 1024 + threadIdx.x; i < n; i += 1024 * gridDim.y)
    qo[i] = val(i) - mu * u[i];
  if (!totals) return;
#pragma unroll 1
  for (int a0 = 0; a0 < n_e; a0 += 4) {
    if (a0 > 0) {                   // electrodes beyond the first four
#pragma unroll
      for (int k = 0; k < 4; ++k) t[k] = w[k] = 0.0;
#pragma unroll 1
      for (int i = threadIdx.x; i < n; i += 1024) {
        const int e = eid[i] - a0;
        const double v = val(i), ui = u[i];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          t[k] += e == k ? v : 0.0;
          w[k] += e == k ? ui : 0.0;
        }
      }
    }
    // wave sums, then thread k < 4 adds electrode a0 + k's 16 wave sums in order
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      t[k] = wave_sum(t[k]);
      w[k] = wave_sum(w[k]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        shq[k][wave] = t[k];
        shq[4 + k][wave] = w[k];
      }
    __syncthreads();
    const int k = threadIdx.x;
    if (k < 4 && a0 + k < n_e) {
      double tt = 0.0, ww = 0.0;
      for (int v = 0; v < 16; ++v) {
        tt += shq[k][v];
        ww += shq[4 + k][v];
      }
      Qe[(size_t)b * n_e + a0 + k] = tt - mu * ww;
    }
    __syncthreads();
  }
}

void launch_finalize(hipStream_t st, int n, int batch, const double* qt, int ldqt, const double* add,
                     const double* u, const double* s_dev, const int* eid, int n_e, double* q,
                     int ldq, double* Qe) {
  const dim3 grid(batch, vector_parts(batch, n));
  if (add)
    hipLaunchKernelGGL(k_finalize<true>, grid, dim3(1024), 0, st, n, qt, ldqt, add, u, s_dev, eid,
                       n_e, q, ldq, Qe);
  else
    hipLaunchKernelGGL(k_finalize<false>, grid, dim3(1024), 0, st, n, qt, ldqt, add, u, s_dev, eid,
                       n_e, q, ldq, Qe);
}


// ---------------------------------------------------------------------------
// Inverse kept as the Cholesky factor (the solves are GEMMs with the factor's
// panels, driven from the host).  Electrode indicators as right-hand-side
// rows, and the quantities of Eqs. 4 and 6 from their solutions
// Y_a = g_a^T A^-1 (A symmetric): u = A^-1 e = sum_a Y_a^T (every atom is in
// one electrode), s = e^T u, and S g_a = Y_a^T - u (e^T Y_a^T) / s, since
// u^T g_a = e^T A^-1 g_a.  One workgroup; every sum in a fixed order.
// ---------------------------------------------------------------------------
__global__ void k_group_indicator(int n, int npad, int rows, const int* __restrict__ eid, int n_e,
                                  double* __restrict__ X) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)rows * npad) return;
  const int r = (int)(e / npad), j = (int)(e % npad);
  X[e] = (r < n_e && j < n && eid[j] == r) ? 1.0 : 0.0;
}

void launch_group_indicator(hipStream_t st, int n, int npad, int rows, const int* eid, int n_e,
                            double* X) {
  const size_t tot = (size_t)rows * npad;
  hipLaunchKernelGGL(k_group_indicator, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n,
                     npad, rows, eid, n_e, X);
}

__global__ void __launch_bounds__(1024) k_factor_response(int n, int npad, int n_e,
                                                          const double* __restrict__ Y, int ldy,
                                                          double* __restrict__ u,
                                                          double* __restrict__ s_out,
                                                          double* __restrict__ sg) {
  __shared__ double sh[16];
  __shared__ double tot[CCM_MAXE];
  for (int a = 0; a < n_e; ++a) {
    double t = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) t += Y[(size_t)a * ldy + i];
    t = block_sum1024(t, sh);
    if (threadIdx.x == 0) tot[a] = t;
  }
  __syncthreads();
  double s = 0.0;
  for (int a = 0; a < n_e; ++a) s += tot[a];           // e^T u
  for (int i = threadIdx.x; i < npad; i += 1024) {
    double ui = 0.0;
    if (i < n)
      for (int a = 0; a < n_e; ++a) ui += Y[(size_t)a * ldy + i];
    u[i] = ui;
    for (int a = 0; a < n_e; ++a)
      sg[(size_t)i * n_e + a] = i < n ? Y[(size_t)a * ldy + i] - ui * (tot[a] / s) : 0.0;
  }
  if (threadIdx.x == 0) *s_out = s;
}

void launch_factor_response(hipStream_t st, int n, int npad, int n_e, const double* Y, int ldy,
                            double* u, double* s, double* sg) {
  hipLaunchKernelGGL(k_factor_response, dim3(1), dim3(1024), 0, st, n, npad, n_e, Y, ldy, u, s, sg);
}

// ---------------------------------------------------------------------------
// Row sums of a symmetric npad x npad matrix over each electrode's columns,
// U = M G (npad x n_e, row-major; rows i >= n are zero), in one pass over M:
// one wave per row, lane-strided columns, one register per electrode and a
// fixed-order wave sum each.  M = A^-1 gives the constrained-charge response
// of Eq. 7; M = S gives the cached potential response S G of Eq. 6.
// ---------------------------------------------------------------------------
template <int NE>
__global__ void __launch_bounds__(256) k_group_row_sums(int n, int npad, const double* __restrict__ M,
                                                        const int* __restrict__ eid, int n_e,
                                                        double* __restrict__ U) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= npad) return;
  double acc[NE];
#pragma unroll
  for (int a = 0; a < NE; ++a) acc[a] = 0.0;
  if (i < n) {
    const double* row = M + (size_t)i * npad;
    for (int j = lane; j < n; j += 64) {
      const double v = row[j];
      const int e = eid[j];
#pragma unroll
      for (int a = 0; a < NE; ++a)
        if (e == a) acc[a] += v;
    }
  }
#pragma unroll
  for (int a = 0; a < NE; ++a) {
    const double s = wave_sum(acc[a]);
    if (lane == 0 && a < n_e) U[(size_t)i * n_e + a] = s;
  }
}

void launch_ccm_response(hipStream_t st, int n, int npad, const double* M, const int* eid,
                         int n_e, double* U) {
  dim3 grid((npad + 3) / 4), block(256);
  if (n_e <= 2)
    hipLaunchKernelGGL(k_group_row_sums<2>, grid, block, 0, st, n, npad, M, eid, n_e, U);
  else if (n_e <= 4)
    hipLaunchKernelGGL(k_group_row_sums<4>, grid, block, 0, st, n, npad, M, eid, n_e, U);
  else if (n_e <= 8)
    hipLaunchKernelGGL(k_group_row_sums<8>, grid, block, 0, st, n, npad, M, eid, n_e, U);
  else
    hipLaunchKernelGGL(k_group_row_sums<CCM_MAXE>, grid, block, 0, st, n, npad, M, eid, n_e, U);
}

// Applied potential from the cached response (Eqs. 5, 6): v_i = v~_e(i) and
// d_i = sum_a (S G)_ia v~_a (fixed electrode order), for i < npad (zero
// padding); d is left alone when SG is NULL (the operator has no S).
__global__ void k_apply_potential(int n, int npad, int n_e, const int* __restrict__ eid,
                                  const double* __restrict__ SG, ElectrodeValues vt,
                                  double* __restrict__ vat, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  double v = 0.0, di = 0.0;
  if (i < n) {
    v = vt.v[eid[i]];
    if (SG)
      for (int a = 0; a < n_e; ++a) di += SG[(size_t)i * n_e + a] * vt.v[a];
  }
  vat[i] = v;
  if (SG) d[i] = di;
}

void launch_apply_potential(hipStream_t st, int n, int npad, int n_e, const int* eid,
                            const double* SG, const ElectrodeValues& vt, double* vat, double* d) {
  hipLaunchKernelGGL(k_apply_potential, dim3((npad + 255) / 256), dim3(256), 0, st, n, npad, n_e,
                     eid, SG, vt, vat, d);
}

// Finite-field potential (Eqs. 13, 14) from its cached pieces: v = -dv0 zeta
// and d = S v = -dv0 (S zeta) (szeta NULL: d untouched).
__global__ void k_scale_field(int npad, double dv0, const double* __restrict__ zeta,
                              const double* __restrict__ szeta, double* __restrict__ vat,
                              double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  vat[i] = -dv0 * zeta[i];
  if (szeta) d[i] = -dv0 * szeta[i];
}

void launch_scale_field(hipStream_t st, int npad, double dv0, const double* zeta,
                        const double* szeta, double* vat, double* d) {
  hipLaunchKernelGGL(k_scale_field, dim3((npad + 255) / 256), dim3(256), 0, st, npad, dv0, zeta,
                     szeta, vat, d);
}

// Per configuration b (one workgroup): y = A^-1 b is given (row b of yt);
// q~_b = G^T y, v~ = C~^-1 (Q - q~_b), q = y + U v~, Qe = G^T q.  Sums per
// electrode in a fixed order; n_e <= CCM_MAXE.
__global__ void __launch_bounds__(256) k_ccm_finalize(int n, const double* __restrict__ yt, int ldy,
                                                      const double* __restrict__ U,
                                                      const double* __restrict__ Cinv,
                                                      const double* __restrict__ Qt,
                                                      const int* __restrict__ eid, int n_e,
                                                      double* __restrict__ q, int ldq,
                                                      double* __restrict__ Qe) {
  __shared__ double sh[4];
  __shared__ double s_v[CCM_MAXE];
  __shared__ double s_g[CCM_MAXE];
  const int b = blockIdx.x;
  const double* y = yt + (size_t)b * ldy;
  for (int a = 0; a < n_e; ++a) {
    double t = 0.0;
    for (int i = threadIdx.x; i < n; i += 256)
      if (eid[i] == a) t += y[i];
    t = block_sum256(t, sh);
    if (threadIdx.x == 0) s_g[a] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int a = 0; a < n_e; ++a) {
      double v = 0.0;
      for (int c = 0; c < n_e; ++c) v += Cinv[a * n_e + c] * (Qt[c] - s_g[c]);
      s_v[a] = v;
    }
  __syncthreads();
  double* qo = q + (size_t)b * ldq;
  for (int i = threadIdx.x; i < n; i += 256) {
    double v = y[i];
    for (int a = 0; a < n_e; ++a) v += U[(size_t)i * n_e + a] * s_v[a];
    qo[i] = v;
  }
  if (Qe) {
    __syncthreads();
    for (int a = 0; a < n_e; ++a) {
      double t = 0.0;
      for (int i = threadIdx.x; i < n; i += 256)
        if (eid[i] == a) t += qo[i];
      t = block_sum256(t, sh);
      if (threadIdx.x == 0) Qe[(size_t)b * n_e + a] = t;
    }
  }
}

void launch_ccm_finalize(hipStream_t st, int n, int batch, const double* yt, int ldy,
                         const double* U, const double* Cinv, const double* Qt, const int* eid,
                         int n_e, double* q, int ldq, double* Qe) {
  hipLaunchKernelGGL(k_ccm_finalize, dim3(batch), dim3(256), 0, st, n, yt, ldy, U, Cinv, Qt, eid,
                     n_e, q, ldq, Qe);
}

// p[0 .. count) = 0 (a kernel, so it can sit inside a captured graph)
__global__ void k_fill_zero(size_t count, float* p) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = 0.0f;
}

void launch_fill_zero(hipStream_t st, size_t count, float* p) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, p);
}

// dst (rows x npad, FP64) = src (batch x n) zero-padded in both directions
__global__ void k_pad_rows(int n, int npad, int batch, int rows, const void* __restrict__ src,
                           int src_is_f32, const double* __restrict__ shift,
                           double* __restrict__ dst) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)rows * npad) return;
  const int r = (int)(e / npad), j = (int)(e % npad);
  double v = 0.0;
  if (r < batch && j < n)
    v = (src_is_f32 ? (double)reinterpret_cast<const float*>(src)[(size_t)r * n + j]
                    : reinterpret_cast<const double*>(src)[(size_t)r * n + j]) -
        (shift ? shift[r] : 0.0);
  dst[e] = v;
}

void launch_pad_rows(hipStream_t st, int n, int npad, int batch, int rows, const void* src,
                     int src_is_f32, const double* shift, double* dst) {
  const size_t tot = (size_t)rows * npad;
  hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, npad,
                     batch, rows, src, src_is_f32, shift, dst);
}

// ---------------------------------------------------------------------------
// Batched solve on BF16 matrix cores: C (+)= X S with both operands split as
// x ~ hi + lo (BF16 pairs) and three products hi*hi + hi*lo + lo*hi
// accumulated in FP32 (the lo*lo term is below FP32 resolution of the sum).
// S is symmetric, so its rows serve as the columns of the right operand and
// both operands are read K-contiguous.
//
// One persistent kernel serves a group of up to GB_MAXP independent
// problems (contexts of different sizes): the tiles of all problems form one
// list that the workgroups walk with a stride of the grid size.  Tile shape
// BM x 64 (BM = 32, 64 or 128 rows of X) and the split of K into ks parts
// are chosen per problem size by the autotuner; with ks > 1 each part
// writes its own slice of a partial buffer and k_sum_ksplit adds the slices
// in a fixed order.  4 waves in a 2 x 2 layout, v_mfma_f32_16x16x32_bf16,
// K slabs of 32 through LDS with the next slab prefetched into registers.
//   operand layout (lane l): A (row l%16, k 8(l/16)..+7); B (k 8(l/16)..+7,
//   col l%16); result register r: (row 4(l/16) + r, col l%16).
// ---------------------------------------------------------------------------
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <int BM>
__global__ void __launch_bounds__(256) k_gemm_bf16x3(GemmGroupBf grp) {
  constexpr int P = 40;                 // LDS row pitch in BF16 elements (32 + 8)
  constexpr int FM = BM / 32;           // 16-row blocks per wave
  __shared__ __attribute__((aligned(16))) uint16_t Ah[BM * P], Al[BM * P], Bh[64 * P], Bl[64 * P];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * 32;
  for (int t = blockIdx.x; t < grp.total; t += gridDim.x) {
    int p = 0;
    while (p + 1 < grp.nprob && t >= grp.start[p + 1]) ++p;
    const GemmProbBf& pr = grp.p[p];
    const int local = t - grp.start[p];
    const int kpart = local % pr.ks, rest = local / pr.ks;
    const int m0 = (rest / pr.tiles_n) * BM, n0 = (rest % pr.tiles_n) * 64;
    const int kchunk = ((pr.K + pr.ks - 1) / pr.ks + 31) / 32 * 32;
    const int kb = kpart * kchunk, ke = min(pr.K, kb + kchunk);
    v4f acc[FM][2];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
    // loader slots: X rows (BM x 32 BF16 hi and lo per slab), S rows (64 x 32)
    const int sr = tid >> 2, sc = (tid & 3) * 8;
    constexpr int XR = BM >= 64 ? BM / 64 : 1;        // 8-element X groups per thread
    uint4 xh[XR], xl[XR];
    uint2 xh2, xl2;                                    // BM = 32: 4 elements per thread
    uint4 sh, sl;
    auto load = [&](int k0) {
      if constexpr (BM >= 64) {
#pragma unroll
        for (int u = 0; u < XR; ++u) {
          const size_t xo = (size_t)(m0 + sr + 64 * u) * pr.ldx + k0 + sc;
          xh[u] = *reinterpret_cast<const uint4*>(pr.Xhi + xo);
          xl[u] = *reinterpret_cast<const uint4*>(pr.Xlo + xo);
        }
      } else {
        const size_t xo = (size_t)(m0 + (tid >> 3)) * pr.ldx + k0 + (tid & 7) * 4;
        xh2 = *reinterpret_cast<const uint2*>(pr.Xhi + xo);
        xl2 = *reinterpret_cast<const uint2*>(pr.Xlo + xo);
      }
      const size_t so = (size_t)(n0 + sr) * pr.lds + k0 + sc;
      sh = *reinterpret_cast<const uint4*>(pr.Shi + so);
      sl = *reinterpret_cast<const uint4*>(pr.Slo + so);
    };
    auto store = [&]() {
      if constexpr (BM >= 64) {
#pragma unroll
        for (int u = 0; u < XR; ++u) {
          *reinterpret_cast<uint4*>(&Ah[(sr + 64 * u) * P + sc]) = xh[u];
          *reinterpret_cast<uint4*>(&Al[(sr + 64 * u) * P + sc]) = xl[u];
        }
      } else {
        const int r = tid >> 3, c4 = (tid & 7) * 4;
        *reinterpret_cast<uint2*>(&Ah[r * P + c4]) = xh2;
        *reinterpret_cast<uint2*>(&Al[r * P + c4]) = xl2;
      }
      *reinterpret_cast<uint4*>(&Bh[sr * P + sc]) = sh;
      *reinterpret_cast<uint4*>(&Bl[sr * P + sc]) = sl;
    };
    if (kb < ke) load(kb);
    for (int k0 = kb; k0 < ke; k0 += 32) {
      __syncthreads();                 // the previous slab (or tile) is no longer read
      store();
      __syncthreads();
      if (k0 + 32 < ke) load(k0 + 32);
      const int kk = 8 * (lane >> 4), rr = lane & 15;
      v8bf ah[FM], al[FM], bh[2], bl[2];
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        ah[a] = *reinterpret_cast<const v8bf*>(&Ah[(wm + a * 16 + rr) * P + kk]);
        al[a] = *reinterpret_cast<const v8bf*>(&Al[(wm + a * 16 + rr) * P + kk]);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        bh[b] = *reinterpret_cast<const v8bf*>(&Bh[(wn + b * 16 + rr) * P + kk]);
        bl[b] = *reinterpret_cast<const v8bf*>(&Bl[(wn + b * 16 + rr) * P + kk]);
      }
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
        }
    }
    // ks == 1: C (+)= result; ks > 1: slice kpart of the partial buffer
    double* out = pr.ks > 1 ? pr.part + (size_t)kpart * pr.M * pr.ldc : pr.C;
    const bool acc_c = pr.ks == 1 && pr.accumulate;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm + a * 16 + 4 * (lane >> 4) + r;
          const int col = n0 + wn + b * 16 + (lane & 15);
          double* cp = out + (size_t)row * pr.ldc + col;
          const double v = (double)acc[a][b][r];
          *cp = acc_c ? *cp + v : v;
        }
  }
}

// C (+)= sum over ks slices of part, in slice order (fixed), M x ldc elements
__global__ void k_sum_ksplit(size_t count, int ks, const double* __restrict__ part,
                             double* __restrict__ C, int accumulate) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double s = part[e];
  for (int k = 1; k < ks; ++k) s += part[(size_t)k * count + e];
  C[e] = accumulate ? C[e] + s : s;
}

void launch_gemm_bf16x3_group(hipStream_t st, const GemmGroupBf& grp, int bm, int grid) {
  if (grp.total <= 0) return;
  const int g = std::max(1, std::min(grid, grp.total));
  if (bm == 32)
    hipLaunchKernelGGL(k_gemm_bf16x3<32>, dim3(g), dim3(256), 0, st, grp);
  else if (bm == 128)
    hipLaunchKernelGGL(k_gemm_bf16x3<128>, dim3(g), dim3(256), 0, st, grp);
  else
    hipLaunchKernelGGL(k_gemm_bf16x3<64>, dim3(g), dim3(256), 0, st, grp);
  for (int p = 0; p < grp.nprob; ++p) {
    const GemmProbBf& pr = grp.p[p];
    if (pr.ks > 1) {
      const size_t count = (size_t)pr.M * pr.ldc;
      hipLaunchKernelGGL(k_sum_ksplit, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                         count, pr.ks, pr.part, pr.C, pr.accumulate);
    }
  }
}

// Fill one problem of a group: X (M x K, ld ldx), S hi/lo (N x K, ld lds),
// C (M x ldc); part: ks x M x ldc doubles when ks > 1.
GemmProbBf gemm_bf16x3_problem(int M, int N, int K, const uint16_t* Xhi, const uint16_t* Xlo,
                               int ldx, const uint16_t* Shi, const uint16_t* Slo, int lds,
                               double* C, int ldc, int accumulate, int bm, int ks, double* part) {
  GemmProbBf pr{};
  pr.Xhi = Xhi; pr.Xlo = Xlo; pr.Shi = Shi; pr.Slo = Slo; pr.C = C; pr.part = part;
  pr.M = M; pr.N = N; pr.K = K; pr.ldx = ldx; pr.lds = lds; pr.ldc = ldc;
  pr.tiles_m = M / bm; pr.tiles_n = N / 64; pr.ks = ks; pr.accumulate = accumulate;
  return pr;
}

void group_finish(GemmGroupBf& grp) {
  grp.start[0] = 0;
  for (int p = 0; p < grp.nprob; ++p)
    grp.start[p + 1] = grp.start[p] + grp.p[p].tiles_m * grp.p[p].tiles_n * grp.p[p].ks;
  grp.total = grp.start[grp.nprob];
}

}  // namespace cpm
