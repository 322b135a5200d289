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
// Structure factors.  One thread per k run (256 runs per workgroup) and a
// chunk of the electrolyte per workgroup, staged in LDS tiles of up to SF_TJ
// charges together with per-charge phase tables
//   tx[n] = q_j e^{2 pi i n fx_j} (n = 0..nxm), ty[n] = e^{2 pi i n fy_j}
//   (n = 0..nym), tz[n] = e^{2 pi i n fz_j} (n = 0..nzm),
// built in segments of SF_SEG entries: an exact FP64 sincospi at the first
// entry, then rotations by e^{2 pi i f}.  Negative indices use the conjugate.
// A run starts at tx[nx] ty[ny] tz[nz0] (two complex products) and advances
// along k_z by tz[1] (FP64 rotation).  Two charges are walked together so
// two independent rotation chains are in flight.  T is the accumulation type.
// part[(chunk * nk + k) * 2 + {0,1}] = partial S(k) over the chunk's charges;
// the workgroups of the first run block also leave the chunk's partial dipole
// sum_j q_j z_j in mz_part[chunk].
// ---------------------------------------------------------------------------
constexpr int SF_TJ = 16;
constexpr int SF_SEG = 8;

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <typename T>
__global__ void __launch_bounds__(256) k_structure_factor(int nruns, const KRun* __restrict__ runs,
                                                          int nk, int m, int chunk_size, int tj,
                                                          const double* __restrict__ xyz,
                                                          const double* __restrict__ q, double Lx,
                                                          double Ly, double Lz, int nxm, int nym,
                                                          int nzm, double* __restrict__ part,
                                                          double* __restrict__ mz_part) {
  extern __shared__ double2 tab[];                  // [tj][W]
  __shared__ double s_f[3][SF_TJ], s_q[SF_TJ];
  __shared__ double2 s_e1[3][SF_TJ];
  __shared__ double s_mz[4];
  const int W = nxm + nym + nzm + 3, oy = nxm + 1, oz = nxm + nym + 2;
  const int nsx = (nxm + SF_SEG) / SF_SEG, nsy = (nym + SF_SEG) / SF_SEG,
            nsz = (nzm + SF_SEG) / SF_SEG, nseg = nsx + nsy + nsz;
  const int rid = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  const int j0 = chunk * chunk_size;
  const int j1 = min(m, j0 + chunk_size);
  KRun run = {0, 0, 0, 0, 0, 0};
  if (rid < nruns) run = runs[rid];
  const int iy = oy + abs(run.ny), iz = oz + abs(run.nz0);
  const double sy = run.ny < 0 ? -1.0 : 1.0, sz0 = run.nz0 < 0 ? -1.0 : 1.0;
  T are[RUN], aim[RUN];
#pragma unroll
  for (int r = 0; r < RUN; ++r) { are[r] = 0; aim[r] = 0; }
  double mz = 0.0;

  for (int jt = j0; jt < j1; jt += tj) {
    const int nt = min(tj, j1 - jt);
    __syncthreads();
    if ((int)threadIdx.x < nt) {
      const int t = threadIdx.x, j = jt + t;
      const double x = xyz[3 * j], y = xyz[3 * j + 1], z = xyz[3 * j + 2];
      const double fx = x / Lx, fy = y / Ly;
      s_f[0][t] = fx - floor(fx);
      s_f[1][t] = fy - floor(fy);
      s_f[2][t] = z / Lz;
      s_q[t] = q[j];
      if (blockIdx.x == 0) mz += q[j] * z;
    }
    __syncthreads();
    if ((int)threadIdx.x < 3 * nt) {
      const int ax = threadIdx.x / nt, t = threadIdx.x - ax * nt;
      const double f = s_f[ax][t];
      double sn, cs;
      sincospi(2.0 * (f - rint(f)), &sn, &cs);
      s_e1[ax][t] = make_double2(cs, sn);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nt * nseg; e += blockDim.x) {
      const int t = e / nseg, sg = e - t * nseg;
      const int ax = sg < nsx ? 0 : (sg < nsx + nsy ? 1 : 2);
      const int s0 = sg - (ax == 0 ? 0 : (ax == 1 ? nsx : nsx + nsy));
      const int nmax = ax == 0 ? nxm : (ax == 1 ? nym : nzm);
      const int off = ax == 0 ? 0 : (ax == 1 ? oy : oz);
      const int n0 = s0 * SF_SEG, n1 = min(nmax, n0 + SF_SEG - 1);
      double th = n0 * s_f[ax][t];
      th -= rint(th);
      double sn, cs;
      sincospi(2.0 * th, &sn, &cs);
      const double sc = ax == 0 ? s_q[t] : 1.0;
      double2 v = make_double2(cs, sn);
      const double2 e1 = s_e1[ax][t];
      double2* dst = tab + t * W + off;
      for (int nn = n0; nn <= n1; ++nn) {
        dst[nn] = make_double2(sc * v.x, sc * v.y);
        v = cmul(v, e1);
      }
    }
    __syncthreads();
    if (rid < nruns) {
      int t = 0;
      for (; t + 1 < nt; t += 2) {
        const double2* ta = tab + t * W;
        const double2* tb = ta + W;
        double2 eya = ta[iy], eza = ta[iz], eyb = tb[iy], ezb = tb[iz];
        eya.y *= sy; eza.y *= sz0; eyb.y *= sy; ezb.y *= sz0;
        double2 wa = cmul(cmul(ta[run.nx], eya), eza);
        double2 wb = cmul(cmul(tb[run.nx], eyb), ezb);
        const double2 sa = ta[oz + 1], sb = tb[oz + 1];
#pragma unroll
        for (int r = 0; r < RUN; ++r) {
          are[r] += (T)(wa.x + wb.x);
          aim[r] += (T)(wa.y + wb.y);
          wa = cmul(wa, sa);
          wb = cmul(wb, sb);
        }
      }
      if (t < nt) {
        const double2* ta = tab + t * W;
        double2 eya = ta[iy], eza = ta[iz];
        eya.y *= sy; eza.y *= sz0;
        double2 wa = cmul(cmul(ta[run.nx], eya), eza);
        const double2 sa = ta[oz + 1];
#pragma unroll
        for (int r = 0; r < RUN; ++r) {
          are[r] += (T)wa.x;
          aim[r] += (T)wa.y;
          wa = cmul(wa, sa);
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
  if (blockIdx.x == 0) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) mz += __shfl_xor(mz, o, 64);
    if (lane == 0) s_mz[wave] = mz;
    __syncthreads();
    if (threadIdx.x == 0) mz_part[chunk] = (s_mz[0] + s_mz[1]) + (s_mz[2] + s_mz[3]);
  }
}

int sf_tile(int nxm, int nym, int nzm) {
  const int W = nxm + nym + nzm + 3;
  int tj = (int)(30720 / (W * sizeof(double2)));   // <= 30 KB of dynamic LDS
  return tj < 1 ? 1 : (tj > SF_TJ ? SF_TJ : tj);
}

void launch_b_structure_factor(hipStream_t st, int fp32, int nruns, const KRun* runs, int nk, int m,
                               int mchunks, const double* xyz, const double* q, double Lx,
                               double Ly, double Lz, int nxm, int nym, int nzm, double* part,
                               double* mz_part) {
  const int chunk_size = (m + mchunks - 1) / mchunks;
  const int tj = sf_tile(nxm, nym, nzm);
  const size_t shm = (size_t)tj * (nxm + nym + nzm + 3) * sizeof(double2);
  dim3 grid((nruns + 255) / 256, mchunks), block(256);
  if (fp32)
    hipLaunchKernelGGL(k_structure_factor<float>, grid, block, shm, st, nruns, runs, nk, m,
                       chunk_size, tj, xyz, q, Lx, Ly, Lz, nxm, nym, nzm, part, mz_part);
  else
    hipLaunchKernelGGL(k_structure_factor<double>, grid, block, shm, st, nruns, runs, nk, m,
                       chunk_size, tj, xyz, q, Lx, Ly, Lz, nxm, nym, nzm, part, mz_part);
}

// sfw[k] = 2 W(k) * sum_chunks part[chunk][k]   (fixed chunk order)
__global__ void k_sf_reduce(int nk, int mchunks, const double* __restrict__ part,
                            const double* __restrict__ w2, double* __restrict__ sfw) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  double re = 0.0, im = 0.0;
#pragma unroll 4
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
// k-space potential at the electrode atoms: one thread per atom, a chunk of
// whole (k_x, k_y) columns per workgroup with the columns' weighted structure
// factors staged in LDS (every lane reads the same k).  Per column the phase
// e^{i k.R_i} is computed once in FP64 (sincospi) and then rotated along k_z
// in FP64; two interleaved sub-sequences (even and odd k_z, rotated by
// e^{2i k_z1 z_i}) keep two independent dependency chains in flight.
// part[chunk * n + i] = sum over the chunk's k of Re[e^{-i k.R_i} 2W S(k)].
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(128) k_kspace_project(int n, const KCol* __restrict__ cols,
                                                        const int* __restrict__ chunk_col,
                                                        const double* __restrict__ fx,
                                                        const double* __restrict__ fy,
                                                        const double* __restrict__ fz,
                                                        const double* __restrict__ sfw,
                                                        double* __restrict__ part) {
  __shared__ double2 s_w[PJ_MAXK];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  const int c0 = chunk_col[chunk], c1 = chunk_col[chunk + 1];
  const int kbase = cols[c0].koff;
  const int kend = cols[c1 - 1].koff + cols[c1 - 1].len;
  for (int t = threadIdx.x; t < kend - kbase; t += blockDim.x)
    s_w[t] = make_double2(sfw[2 * (kbase + t)], sfw[2 * (kbase + t) + 1]);
  __syncthreads();
  if (i >= n) return;
  const double ax = fx[i], ay = fy[i], az = fz[i];
  double s1, c1d, s2, c2d;
  sincospi(2.0 * (az - rint(az)), &s1, &c1d);
  const double a2 = 2.0 * az;
  sincospi(2.0 * (a2 - rint(a2)), &s2, &c2d);
  const double2 z2 = make_double2(c2d, s2);
  const double2 z1 = make_double2(c1d, s1);
  T acc0 = 0, acc1 = 0;
  for (int c = c0; c < c1; ++c) {
    const KCol col = cols[c];
    double th = col.nx * ax + col.ny * ay + col.lo * az;
    th -= rint(th);
    double sn, cs;
    sincospi(2.0 * th, &sn, &cs);
    double2 e0 = make_double2(cs, sn);           // k_z = lo, lo + 2, ...
    double2 e1 = cmul(e0, z1);                   // k_z = lo + 1, lo + 3, ...
    const double2* w = s_w + (col.koff - kbase);
    int r = 0;
    for (; r + 1 < col.len; r += 2) {
      acc0 += (T)(e0.x * w[r].x + e0.y * w[r].y);
      acc1 += (T)(e1.x * w[r + 1].x + e1.y * w[r + 1].y);
      e0 = cmul(e0, z2);
      e1 = cmul(e1, z2);
    }
    if (r < col.len) acc0 += (T)(e0.x * w[r].x + e0.y * w[r].y);
  }
  part[(size_t)chunk * n + i] = (double)acc0 + (double)acc1;
}

void launch_b_kspace_project(hipStream_t st, int fp32, int n, int kchunks, const KCol* cols,
                             const int* chunk_col, const Buffers& b, const double* sfw,
                             double* part) {
  dim3 grid((n + 127) / 128, kchunks), block(128);
  if (fp32)
    hipLaunchKernelGGL(k_kspace_project<float>, grid, block, 0, st, n, cols, chunk_col, b.efx,
                       b.efy, b.efz, sfw, part);
  else
    hipLaunchKernelGGL(k_kspace_project<double>, grid, block, 0, st, n, cols, chunk_col, b.efx,
                       b.efy, b.efz, sfw, part);
}

// ---------------------------------------------------------------------------
// Real-space pair sum: one thread per electrode atom, electrolyte tiles in LDS.
// part[chunk * n + i] = sum_j q_j sum_t [erfc(alpha r) - erfc(eta r)] / r.
// ---------------------------------------------------------------------------
constexpr int RS_TILE = 256;

// erfc(alpha r) - erfc(eta r).  Beyond r2_gauss = 45 / (eta^2 - alpha^2) the
// second term is below e^-45 of the first (erfc(x) <= e^{-x^2}), i.e. under
// FP64 rounding of the difference, and is not evaluated.
__device__ inline double pair_kernel(double r, double r2, double alpha, double eta,
                                     double r2_gauss) {
  const double a = erfc(alpha * r);
  return r2 > r2_gauss ? a : a - erfc(eta * r);
}

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
  const double r2_gauss = eta > alpha ? 45.0 / (eta * eta - alpha * alpha) : 1e300;
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
          if (r < rc) acc += s_q[t] * pair_kernel(r, r2, alpha, eta, r2_gauss) / r;
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
              if (r < rc) acc += s_q[t] * pair_kernel(r, r2, alpha, eta, r2_gauss) / r;
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

// b_i = -k_e (sum of k-space partials + sum of real-space partials + (4 pi/V) z_i M_z)
__global__ void k_combine(int n, int kchunks, int rchunks, int mchunks,
                          const double* __restrict__ phik, const double* __restrict__ phir,
                          const double* __restrict__ ez, const double* __restrict__ mz_part,
                          double slab_coef, double ke, void* out, int out_is_f32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // fixed-order sums; the loads are independent, so unrolling keeps many in flight
  double pk = 0.0, pr = 0.0;
#pragma unroll 8
  for (int c = 0; c < kchunks; ++c) pk += phik[(size_t)c * n + i];
#pragma unroll 8
  for (int c = 0; c < rchunks; ++c) pr += phir[(size_t)c * n + i];
  double mz = 0.0;
  for (int c = 0; c < mchunks; ++c) mz += mz_part[c];
  const double b = -ke * (pk + pr + slab_coef * ez[i] * mz);
  if (out_is_f32)
    reinterpret_cast<float*>(out)[i] = (float)b;
  else
    reinterpret_cast<double*>(out)[i] = b;
}

void launch_b_combine(hipStream_t st, int n, int kchunks, int rchunks, int mchunks,
                      const double* phik, const double* phir, const Buffers& b,
                      const double* mz_part, double slab_coef, double ke, void* out,
                      int out_is_f32) {
  hipLaunchKernelGGL(k_combine, dim3((n + 63) / 64), dim3(64), 0, st, n, kchunks, rchunks, mchunks,
                     phik, phir, b.ez, mz_part, slab_coef, ke, out, out_is_f32);
}

}  // namespace cpm
