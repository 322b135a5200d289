// The electrolyte vector b, recomputed for every electrolyte configuration
// (ELECTRODE paper, Sec. II.A: "the main computational burden").  b is minus
// the electrolyte potential at the Gaussian electrode atoms:
//
//   b_i = -k_e { sum_j q_j sum_t [erfc(alpha r) - erfc(eta r)] / r     (real space)
//              + sum_{k in K+} 2 W(k) Re[ e^{-i k.R_i} S(k) ]           (k space)
//              + (4 pi / V) z_i M_z }                                   (slab, Eq. 12)
//
// with the structure factor S(k) = sum_j q_j e^{i k.r_j} and the electrolyte
// dipole M_z = sum_j q_j z_j.  The neutral electrolyte makes the k = 0
// background term vanish.
//
// The k set is walked in runs of up to RUN consecutive k_z in one (k_x, k_y)
// column.  The phase at the start of a run is computed exactly in FP64 from
// fractional coordinates (reduced to [-1/2, 1/2] turns, then sincospi); the
// rest of the run follows by multiplying with e^{2 pi i z / Lz}.  Only the
// accumulation type changes between the FP64 and FP32 variants.
//
// Every sum is split into fixed chunks whose partials are added in a fixed
// order, so results are bitwise reproducible.
#include "cpm_internal.h"

namespace cpm {

// ---------------------------------------------------------------------------
// Structure factors: one thread per k run, electrolyte staged in LDS tiles.
// part[(chunk * nk + k) * 2 + {0,1}] = partial S(k) over the chunk's charges.
// ---------------------------------------------------------------------------
constexpr int SF_TILE = 256;

template <typename T>
__global__ void __launch_bounds__(256) k_structure_factor(int nruns, const KRun* __restrict__ runs,
                                                          int nk, int m, int chunk_size,
                                                          const double* __restrict__ xyz,
                                                          const double* __restrict__ q, double Lx,
                                                          double Ly, double Lz,
                                                          double* __restrict__ part) {
  __shared__ double s_fx[SF_TILE], s_fy[SF_TILE], s_fz[SF_TILE], s_q[SF_TILE];
  __shared__ T s_cz[SF_TILE], s_sz[SF_TILE];
  const int rid = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  const int j0 = chunk * chunk_size;
  const int j1 = min(m, j0 + chunk_size);
  KRun run = {0, 0, 0, 0, 0, 0};
  if (rid < nruns) run = runs[rid];
  T are[RUN], aim[RUN];
#pragma unroll
  for (int r = 0; r < RUN; ++r) { are[r] = 0; aim[r] = 0; }

  for (int jt = j0; jt < j1; jt += SF_TILE) {
    const int nt = min(SF_TILE, j1 - jt);
    __syncthreads();
    if ((int)threadIdx.x < nt) {
      const int j = jt + threadIdx.x;
      double fx = xyz[3 * j] / Lx, fy = xyz[3 * j + 1] / Ly, fz = xyz[3 * j + 2] / Lz;
      fx -= floor(fx);
      fy -= floor(fy);
      s_fx[threadIdx.x] = fx; s_fy[threadIdx.x] = fy; s_fz[threadIdx.x] = fz;
      s_q[threadIdx.x] = q[j];
      double sz, cz;
      sincospi(2.0 * (fz - rint(fz)), &sz, &cz);
      s_cz[threadIdx.x] = (T)cz; s_sz[threadIdx.x] = (T)sz;
    }
    __syncthreads();
    if (rid < nruns) {
      for (int t = 0; t < nt; ++t) {
        double th = run.nx * s_fx[t] + run.ny * s_fy[t] + run.nz0 * s_fz[t];
        th -= rint(th);
        double sn, cs;
        sincospi(2.0 * th, &sn, &cs);
        const double qq = s_q[t];
        T wr = (T)(qq * cs), wi = (T)(qq * sn);
        const T cz = s_cz[t], sz = s_sz[t];
#pragma unroll
        for (int r = 0; r < RUN; ++r) {
          are[r] += wr;
          aim[r] += wi;
          const T nr = wr * cz - wi * sz;
          wi = wr * sz + wi * cz;
          wr = nr;
        }
      }
    }
  }
  if (rid < nruns) {
    double* out = part + ((size_t)chunk * nk + run.koff) * 2;
    for (int r = 0; r < run.len; ++r) {
      out[2 * r] = (double)are[r];
      out[2 * r + 1] = (double)aim[r];
    }
  }
}

void launch_b_structure_factor(hipStream_t st, int fp32, int nruns, const KRun* runs, int nk, int m,
                               int mchunks, const double* xyz, const double* q, double Lx,
                               double Ly, double Lz, double* part) {
  const int chunk_size = (m + mchunks - 1) / mchunks;
  dim3 grid((nruns + 255) / 256, mchunks), block(256);
  if (fp32)
    hipLaunchKernelGGL(k_structure_factor<float>, grid, block, 0, st, nruns, runs, nk, m,
                       chunk_size, xyz, q, Lx, Ly, Lz, part);
  else
    hipLaunchKernelGGL(k_structure_factor<double>, grid, block, 0, st, nruns, runs, nk, m,
                       chunk_size, xyz, q, Lx, Ly, Lz, part);
}

// sfw[k] = 2 W(k) * sum_chunks part[chunk][k]   (fixed chunk order)
__global__ void k_sf_reduce(int nk, int mchunks, const double* __restrict__ part,
                            const double* __restrict__ w2, double* __restrict__ sfw) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < mchunks; ++c) {
    re += part[((size_t)c * nk + k) * 2];
    im += part[((size_t)c * nk + k) * 2 + 1];
  }
  sfw[2 * k] = w2[k] * re;
  sfw[2 * k + 1] = w2[k] * im;
}

void launch_b_sf_reduce(hipStream_t st, int nk, int mchunks, const double* part, const double* w2,
                        double* sfw) {
  hipLaunchKernelGGL(k_sf_reduce, dim3((nk + 255) / 256), dim3(256), 0, st, nk, mchunks, part, w2,
                     sfw);
}

// ---------------------------------------------------------------------------
// k-space potential at the electrode atoms: one thread per atom, the chunk's
// weighted structure factors staged in LDS (every lane reads the same k).
// part[chunk * n + i] = sum over the chunk's k of Re[e^{-i k.R_i} 2W S(k)].
// ---------------------------------------------------------------------------
constexpr int PJ_MAXK = 64 * RUN;      // k values staged per chunk (runs_per_chunk <= 64)

template <typename T>
__global__ void __launch_bounds__(256) k_kspace_project(int n, int nruns, int runs_per_chunk,
                                                        const KRun* __restrict__ runs,
                                                        const double* __restrict__ fx,
                                                        const double* __restrict__ fy,
                                                        const double* __restrict__ fz,
                                                        const double* __restrict__ sfw,
                                                        double* __restrict__ part) {
  __shared__ KRun s_runs[64];
  __shared__ T s_re[PJ_MAXK], s_im[PJ_MAXK];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  const int r0 = chunk * runs_per_chunk;
  const int r1 = min(nruns, r0 + runs_per_chunk);
  if (r0 >= r1) return;
  const int kbase = runs[r0].koff;
  const int kend = runs[r1 - 1].koff + runs[r1 - 1].len;
  for (int t = threadIdx.x; t < r1 - r0; t += blockDim.x) s_runs[t] = runs[r0 + t];
  for (int t = threadIdx.x; t < kend - kbase; t += blockDim.x) {
    s_re[t] = (T)sfw[2 * (kbase + t)];
    s_im[t] = (T)sfw[2 * (kbase + t) + 1];
  }
  __syncthreads();
  if (i >= n) return;
  const double ax = fx[i], ay = fy[i], az = fz[i];
  double szd, czd;
  sincospi(2.0 * (az - rint(az)), &szd, &czd);
  const T cz = (T)czd, sz = (T)szd;
  T acc = 0;
  for (int rr = 0; rr < r1 - r0; ++rr) {
    const KRun run = s_runs[rr];
    double th = run.nx * ax + run.ny * ay + run.nz0 * az;
    th -= rint(th);
    double sn, cs;
    sincospi(2.0 * th, &sn, &cs);
    T er = (T)cs, ei = (T)sn;
    const int kb = run.koff - kbase;
    for (int r = 0; r < run.len; ++r) {
      acc += er * s_re[kb + r] + ei * s_im[kb + r];
      const T nr = er * cz - ei * sz;
      ei = er * sz + ei * cz;
      er = nr;
    }
  }
  part[(size_t)chunk * n + i] = (double)acc;
}

void launch_b_kspace_project(hipStream_t st, int fp32, int n, int nruns, int kchunks,
                             int runs_per_chunk, const KRun* runs, const Buffers& b,
                             const double* sfw, double* part) {
  dim3 grid((n + 255) / 256, kchunks), block(256);
  if (fp32)
    hipLaunchKernelGGL(k_kspace_project<float>, grid, block, 0, st, n, nruns, runs_per_chunk, runs,
                       b.efx, b.efy, b.efz, sfw, part);
  else
    hipLaunchKernelGGL(k_kspace_project<double>, grid, block, 0, st, n, nruns, runs_per_chunk,
                       runs, b.efx, b.efy, b.efz, sfw, part);
}

// ---------------------------------------------------------------------------
// Real-space pair sum: one thread per electrode atom, electrolyte tiles in LDS.
// part[chunk * n + i] = sum_j q_j sum_t [erfc(alpha r) - erfc(eta r)] / r.
// ---------------------------------------------------------------------------
constexpr int RS_TILE = 256;

__global__ void __launch_bounds__(256) k_real_space_b(int n, int m, int chunk_size,
                                                      const double* __restrict__ ex,
                                                      const double* __restrict__ ey,
                                                      const double* __restrict__ ez,
                                                      const double* __restrict__ xyz,
                                                      const double* __restrict__ q, double Lx,
                                                      double Ly, double rc, double alpha,
                                                      double eta, double* __restrict__ part) {
  __shared__ double s_x[RS_TILE], s_y[RS_TILE], s_z[RS_TILE], s_q[RS_TILE];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  const int j0 = chunk * chunk_size, j1 = min(m, j0 + chunk_size);
  const double invLx = 1.0 / Lx, invLy = 1.0 / Ly, rc2 = rc * rc;
  const bool single = (Lx >= 2.0 * rc) && (Ly >= 2.0 * rc);
  double xi = 0, yi = 0, zi = 0;
  if (i < n) { xi = ex[i]; yi = ey[i]; zi = ez[i]; }
  double acc = 0.0;
  for (int jt = j0; jt < j1; jt += RS_TILE) {
    const int nt = min(RS_TILE, j1 - jt);
    __syncthreads();
    if ((int)threadIdx.x < nt) {
      const int j = jt + threadIdx.x;
      double x = xyz[3 * j], y = xyz[3 * j + 1];
      x -= Lx * floor(x * invLx);
      y -= Ly * floor(y * invLy);
      s_x[threadIdx.x] = x; s_y[threadIdx.x] = y; s_z[threadIdx.x] = xyz[3 * j + 2];
      s_q[threadIdx.x] = q[j];
    }
    __syncthreads();
    if (i >= n) continue;
    for (int t = 0; t < nt; ++t) {
      const double dz = zi - s_z[t];
      if (fabs(dz) >= rc) continue;
      double dx = xi - s_x[t], dy = yi - s_y[t];
      dx -= Lx * rint(dx * invLx);
      dy -= Ly * rint(dy * invLy);
      if (single) {
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < rc2 * (1.0 + 1e-12)) {
          const double r = sqrt(r2);
          if (r < rc) acc += s_q[t] * (erfc(alpha * r) - erfc(eta * r)) / r;
        }
      } else {
        const int alo = (int)ceil((-rc - dx) * invLx) - 1, ahi = (int)floor((rc - dx) * invLx) + 1;
        const int blo = (int)ceil((-rc - dy) * invLy) - 1, bhi = (int)floor((rc - dy) * invLy) + 1;
        for (int a = alo; a <= ahi; ++a) {
          const double X = dx + a * Lx;
          for (int bb = blo; bb <= bhi; ++bb) {
            const double Y = dy + bb * Ly;
            const double r2 = X * X + Y * Y + dz * dz;
            if (r2 < rc2 * (1.0 + 1e-12)) {
              const double r = sqrt(r2);
              if (r < rc) acc += s_q[t] * (erfc(alpha * r) - erfc(eta * r)) / r;
            }
          }
        }
      }
    }
  }
  if (i < n) part[(size_t)chunk * n + i] = acc;
}

void launch_b_real_space(hipStream_t st, int n, int m, int rchunks, const Buffers& b,
                         const double* xyz, const double* q, double Lx, double Ly, double rc,
                         double alpha, double eta, double* part) {
  const int chunk_size = (m + rchunks - 1) / rchunks;
  dim3 grid((n + 255) / 256, rchunks), block(256);
  hipLaunchKernelGGL(k_real_space_b, grid, block, 0, st, n, m, chunk_size, b.ex, b.ey, b.ez, xyz, q,
                     Lx, Ly, rc, alpha, eta, part);
}

// M_z = sum_j q_j z_j in one workgroup, fixed order.
__global__ void __launch_bounds__(256) k_dipole(int m, const double* __restrict__ xyz,
                                                const double* __restrict__ q, double* mz) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int j = threadIdx.x; j < m; j += 256) s += q[j] * xyz[3 * j + 2];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *mz = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

void launch_b_dipole(hipStream_t st, int m, const double* xyz, const double* q, double* mz) {
  hipLaunchKernelGGL(k_dipole, dim3(1), dim3(256), 0, st, m, xyz, q, mz);
}

// b_i = -k_e (sum of k-space partials + sum of real-space partials + (4 pi/V) z_i M_z)
__global__ void k_combine(int n, int kchunks, int rchunks, const double* __restrict__ phik,
                          const double* __restrict__ phir, const double* __restrict__ ez,
                          const double* __restrict__ mz, double slab_coef, double ke, void* out,
                          int out_is_f32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double pk = 0.0, pr = 0.0;
  for (int c = 0; c < kchunks; ++c) pk += phik[(size_t)c * n + i];
  for (int c = 0; c < rchunks; ++c) pr += phir[(size_t)c * n + i];
  const double b = -ke * (pk + pr + slab_coef * ez[i] * (*mz));
  if (out_is_f32)
    reinterpret_cast<float*>(out)[i] = (float)b;
  else
    reinterpret_cast<double*>(out)[i] = b;
}

void launch_b_combine(hipStream_t st, int n, int kchunks, int rchunks, const double* phik,
                      const double* phir, const Buffers& b, const double* mz, double slab_coef,
                      double ke, void* out, int out_is_f32) {
  hipLaunchKernelGGL(k_combine, dim3((n + 255) / 256), dim3(256), 0, st, n, kchunks, rchunks, phik,
                     phir, b.ez, mz, slab_coef, ke, out, out_is_f32);
}

}  // namespace cpm
