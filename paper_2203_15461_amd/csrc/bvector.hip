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

// ---------------------------------------------------------------------------
// Structure factors on FP64 matrix cores.  For a (k_x, k_y) column c,
//   S(c, +-n) = sum_j C_cj (Zr_jn +- i Zi_jn),  C_cj = q_j e^{i(k_x x_j + k_y y_j)},
//   Z_jn = e^{2 pi i n z_j / Lz},  n >= 0,
// so with rows (Re C_c, Im C_c) and columns (Zr_n, Zi_n) one real GEMM over
// the charges gives Pr, Qr, Pi, Qi and both S(c, n) = (Pr - Qi) + i (Pi + Qr)
// and S(c, -n) = (Pr + Qi) + i (Pi - Qr).  Columns are sorted by their k_z
// extent and grouped 16 per M tile (32 rows).  A workgroup takes one M tile,
// one half of its n range and one chunk of the electrolyte; each of its waves
// walks its own tiles of 16 charges (no workgroup barrier inside the loop):
// it writes C for its charges and the first 8 phases e^{2 pi i n fz} of its
// n range into a wave-private LDS area (exact FP64 sincospi), then runs
// v_mfma_f64_16x16x4f64 with the B operand advanced in registers by
// e^{2 pi i 8 fz} per 16-wide block.  The 4 waves are summed in a fixed order.
// part[((chunk * mtiles + mt) * 32 + row) * npadc + col]: this chunk's sums.
// ---------------------------------------------------------------------------
typedef double v4d_t __attribute__((ext_vector_type(4)));
constexpr int SFM_TJ = 16;             // charges per wave tile (4 MFMA k-steps)
constexpr int SFM_NB = 4;              // max 16-wide n blocks per workgroup (a third of a tile)
constexpr int SFM_SPLIT = 3;           // workgroups per M tile along n
constexpr int SFM_COLS = 16;           // columns per M tile (32 GEMM rows)

struct SfmWave {                        // wave-private LDS area
  double C[2 * SFM_COLS][SFM_TJ + 1];  // A operand rows (Re C, Im C) x charges
  double2 z0[SFM_TJ][8];               // e^{2 pi i (n_lo + j) fz_t}, j = 0..7
  double2 r8[SFM_TJ];                  // e^{2 pi i 8 fz_t}
};

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(256) k_sf_mfma(int m, int chunk_size, int mtiles,
                                                 const int* __restrict__ sc_nx,
                                                 const int* __restrict__ sc_ny,
                                                 const int* __restrict__ tile_nb, int ncolsort,
                                                 const double* __restrict__ xyz,
                                                 const double* __restrict__ q, double Lx,
                                                 double Ly, double Lz, int npadc,
                                                 double* __restrict__ part,
                                                 double* __restrict__ mz_part) {
  __shared__ SfmWave wl[4];
  __shared__ double red[64 * 2 * SFM_NB * 4];      // one wave's accumulators
  __shared__ int s_nx[SFM_COLS], s_ny[SFM_COLS];
  __shared__ double s_mz[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mt = blockIdx.x / SFM_SPLIT, part_n = blockIdx.x % SFM_SPLIT;
  const int chunk = blockIdx.y;
  const int nbt = tile_nb[mt];
  const int nb_lo = (nbt * part_n) / SFM_SPLIT;
  const int nb_hi = (nbt * (part_n + 1)) / SFM_SPLIT;
  const int nbw = nb_hi - nb_lo;                   // blocks of this workgroup (<= SFM_NB)
  const int n_lo = nb_lo * 8;                      // first complex n of this workgroup
  const int c_base = mt * SFM_COLS;
  const int ncol = min(SFM_COLS, ncolsort - c_base);
  if (tid < SFM_COLS) {
    s_nx[tid] = tid < ncol ? sc_nx[c_base + tid] : 0;
    s_ny[tid] = tid < ncol ? sc_ny[c_base + tid] : 0;
  }
  __syncthreads();
  const int j0 = chunk * chunk_size, j1 = min(m, j0 + chunk_size);
  SfmWave& W = wl[wave];
  v4d_t acc0[SFM_NB], acc1[SFM_NB];
#pragma unroll
  for (int b = 0; b < SFM_NB; ++b) {
    acc0[b] = (v4d_t){0.0, 0.0, 0.0, 0.0};
    acc1[b] = (v4d_t){0.0, 0.0, 0.0, 0.0};
  }
  double mz = 0.0;
  const int t_l = lane & 15, g_l = lane >> 4;     // this lane's charge in the tile, lane group
  for (int jt = j0 + wave * SFM_TJ; jt < j1; jt += 4 * SFM_TJ) {
    const int nt = min(SFM_TJ, j1 - jt);
    double fx = 0.0, fy = 0.0, fz = 0.0, qq = 0.0;
    if (t_l < nt) {
      const int j = jt + t_l;
      fx = xyz[3 * j] / Lx;
      fy = xyz[3 * j + 1] / Ly;
      fz = xyz[3 * j + 2] / Lz;
      fx -= floor(fx);
      fy -= floor(fy);
      qq = q[j];
      if (blockIdx.x == 0 && g_l == 0) mz += qq * xyz[3 * j + 2];
    }
    // A operand: C for columns g_l, g_l + 4, g_l + 8, g_l + 12 of charge t_l,
    // and the first phases of the n range (j = 2 g_l, 2 g_l + 1); the seven
    // independent sincospi are written out so their chains interleave
    {
      double th[7];
#pragma unroll
      for (int u = 0; u < 4; ++u) th[u] = s_nx[g_l + 4 * u] * fx + s_ny[g_l + 4 * u] * fy;
      th[4] = (n_lo + 2 * g_l) * fz;
      th[5] = (n_lo + 2 * g_l + 1) * fz;
      th[6] = 8.0 * fz;
      double sn[7], cs[7];
#pragma unroll
      for (int u = 0; u < 7; ++u) sincospi(2.0 * (th[u] - rint(th[u])), &sn[u], &cs[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int cl = g_l + 4 * u;
        const bool ok = cl < ncol;
        W.C[2 * cl][t_l] = ok ? qq * cs[u] : 0.0;
        W.C[2 * cl + 1][t_l] = ok ? qq * sn[u] : 0.0;
      }
      W.z0[t_l][2 * g_l] = make_double2(cs[4], sn[4]);
      W.z0[t_l][2 * g_l + 1] = make_double2(cs[5], sn[5]);
      if (g_l == 0) W.r8[t_l] = make_double2(cs[6], sn[6]);
    }
    wave_lds_sync();
#pragma unroll 1
    for (int ks = 0; ks < SFM_TJ / 4; ++ks) {
      const int kc = 4 * ks + g_l;                    // k index (charge) of this lane's operands
      const double a0 = W.C[t_l][kc];                 // rows 0..15
      const double a1 = W.C[16 + t_l][kc];            // rows 16..31
      double2 z = W.z0[kc][t_l >> 1];
      const double2 r8 = W.r8[kc];
      const bool im = t_l & 1;
#pragma unroll
      for (int b = 0; b < SFM_NB; ++b) {
        if (b < nbw) {
          const double bv = im ? z.y : z.x;
          acc0[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bv, acc0[b], 0, 0, 0);
          acc1[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv, acc1[b], 0, 0, 0);
          z = cmul(z, r8);
        }
      }
    }
    wave_lds_sync();
  }
  // fixed-order sum of the waves' accumulators (3 + 2 + 1 into wave 0)
  for (int src = 3; src >= 1; --src) {
    __syncthreads();
    if (wave == src)
#pragma unroll
      for (int b = 0; b < SFM_NB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          red[((0 * SFM_NB + b) * 4 + r) * 64 + lane] = acc0[b][r];
          red[((1 * SFM_NB + b) * 4 + r) * 64 + lane] = acc1[b][r];
        }
    __syncthreads();
    if (wave == 0)
#pragma unroll
      for (int b = 0; b < SFM_NB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          acc0[b][r] += red[((0 * SFM_NB + b) * 4 + r) * 64 + lane];
          acc1[b][r] += red[((1 * SFM_NB + b) * 4 + r) * 64 + lane];
        }
  }
  if (wave == 0) {
    // result register r of lane l: row (l >> 4) + 4 r, column l & 15 of block b
    double* out = part + ((size_t)chunk * mtiles + mt) * 32 * (size_t)npadc;
#pragma unroll
    for (int b = 0; b < SFM_NB; ++b) {
      if (b >= nbw) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (lane >> 4) + 4 * r;
        const int col = 16 * (nb_lo + b) + (lane & 15);
        out[(size_t)row * npadc + col] = acc0[b][r];
        out[(size_t)(16 + row) * npadc + col] = acc1[b][r];
      }
    }
  }
  if (blockIdx.x == 0) {   // this chunk's electrolyte dipole sum_j q_j z_j
    for (int o = 32; o > 0; o >>= 1) mz += __shfl_xor(mz, o, 64);
    if (lane == 0) s_mz[wave] = mz;
    __syncthreads();
    if (tid == 0) mz_part[chunk] = (s_mz[0] + s_mz[1]) + (s_mz[2] + s_mz[3]);
  }
}

void launch_b_sf_mfma(hipStream_t st, int m, int mchunks, int mtiles, const int* sc_nx,
                      const int* sc_ny, const int* tile_nb, int ncolsort, const double* xyz,
                      const double* q, double Lx, double Ly, double Lz, int nxm, int nym,
                      int npadc, double* part, double* mz_part) {
  (void)nxm; (void)nym;
  const int chunk_size = (m + mchunks - 1) / mchunks;
  dim3 grid(SFM_SPLIT * mtiles, mchunks), block(256);
  hipLaunchKernelGGL(k_sf_mfma, grid, block, 0, st, m, chunk_size, mtiles, sc_nx, sc_ny, tile_nb,
                     ncolsort, xyz, q, Lx, Ly, Lz, npadc, part, mz_part);
}

// Sum the chunks of the matrix-core structure factors and scatter them to
// the flat k order: thread per (sorted column, n >= 0); sfw = 2W S.
__global__ void k_sf_mfma_reduce(int ncolsort, int mtiles, int mchunks, int npadc,
                                 const int* __restrict__ sc_lo, const int* __restrict__ sc_len,
                                 const int* __restrict__ sc_koff, const int* __restrict__ sc_n0,
                                 const double* __restrict__ part, const double* __restrict__ w2,
                                 double* __restrict__ sfw, const int* __restrict__ n_index) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_index[ncolsort]) return;
  // binary search of the column owning entry e
  int lo = 0, hi = ncolsort;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (n_index[mid] <= e) lo = mid; else hi = mid;
  }
  const int c = lo, n = e - n_index[c] + sc_n0[c];
  const int mt = c / SFM_COLS, cl = c % SFM_COLS;
  double pr = 0, qr = 0, pi = 0, qi = 0;
#pragma unroll 4
  for (int ch = 0; ch < mchunks; ++ch) {
    const double* base = part + ((size_t)ch * mtiles + mt) * 32 * (size_t)npadc;
    pr += base[(size_t)(2 * cl) * npadc + 2 * n];
    qr += base[(size_t)(2 * cl) * npadc + 2 * n + 1];
    pi += base[(size_t)(2 * cl + 1) * npadc + 2 * n];
    qi += base[(size_t)(2 * cl + 1) * npadc + 2 * n + 1];
  }
  const int clo = sc_lo[c], chi = sc_lo[c] + sc_len[c] - 1;
  if (n >= clo && n <= chi) {
    const int k = sc_koff[c] + (n - clo);
    sfw[2 * k] = w2[k] * (pr - qi);
    sfw[2 * k + 1] = w2[k] * (pi + qr);
  }
  if (n > 0 && -n >= clo && -n <= chi) {
    const int k = sc_koff[c] + (-n - clo);
    sfw[2 * k] = w2[k] * (pr + qi);
    sfw[2 * k + 1] = w2[k] * (pi - qr);
  }
}

void launch_b_sf_mfma_reduce(hipStream_t st, int ncolsort, int mtiles, int mchunks, int npadc,
                             const int* sc_lo, const int* sc_len, const int* sc_koff,
                             const int* sc_n0, const int* n_index, int n_total,
                             const double* part, const double* w2, double* sfw) {
  hipLaunchKernelGGL(k_sf_mfma_reduce, dim3((n_total + 255) / 256), dim3(256), 0, st, ncolsort,
                     mtiles, mchunks, npadc, sc_lo, sc_len, sc_koff, sc_n0, part, w2, sfw,
                     n_index);
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
// k-space potential for electrodes made of a few planes of equal z (planar
// electrodes).  With theta = k_x x + k_y y the k-space sum factorises exactly:
//   phi_i = sum_cols Re[ e^{-i theta_c(R_i)} T(c, z_i) ],
//   T(c, z) = sum_{k_z in c} 2W(k) S(k) e^{-i k_z z},
// so T is formed once per (column, plane) and the per-atom work drops from
// |K+| to the number of columns.
// ---------------------------------------------------------------------------
// One wave per column: lanes take k_z values, each phase e^{-i k_z z_L} is
// computed exactly (sincospi), and a fixed-order wave reduction forms
// T(c, L) for every plane L.
__global__ void __launch_bounds__(64) k_layer_sum(int ncols, int nlayers,
                                                  const KCol* __restrict__ cols,
                                                  const double* __restrict__ layer_fz,
                                                  const double* __restrict__ sfw,
                                                  double2* __restrict__ T) {
  const int c = blockIdx.x, lane = threadIdx.x;
  const KCol col = cols[c];
  for (int L = 0; L < nlayers; ++L) {
    const double fz = layer_fz[L];
    double tr = 0.0, ti = 0.0;
    for (int r = lane; r < col.len; r += 64) {
      double th = (col.lo + r) * fz;
      th -= rint(th);
      double sn, cs;
      sincospi(2.0 * th, &sn, &cs);
      const double wr = sfw[2 * (col.koff + r)], wi = sfw[2 * (col.koff + r) + 1];
      // e^{-i k_z z} * (wr + i wi)
      tr += cs * wr + sn * wi;
      ti += cs * wi - sn * wr;
    }
    for (int o = 32; o > 0; o >>= 1) {
      tr += __shfl_xor(tr, o, 64);
      ti += __shfl_xor(ti, o, 64);
    }
    if (lane == 0) T[(size_t)c * nlayers + L] = make_double2(tr, ti);
  }
}

constexpr int LP_COLS = 32;           // columns per projection chunk (layer path)

__global__ void __launch_bounds__(64) k_layer_project(int n, int ncols, int nlayers,
                                                      const KCol* __restrict__ cols,
                                                      const int* __restrict__ layer_of,
                                                      const double* __restrict__ fx,
                                                      const double* __restrict__ fy,
                                                      const double2* __restrict__ T,
                                                      double* __restrict__ part) {
  __shared__ int s_nx[LP_COLS], s_ny[LP_COLS];
  __shared__ double2 s_T[LP_COLS * MAX_LAYERS];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  const int c0 = chunk * LP_COLS, c1 = min(ncols, c0 + LP_COLS);
  for (int t = threadIdx.x; t < c1 - c0; t += blockDim.x) {
    s_nx[t] = cols[c0 + t].nx;
    s_ny[t] = cols[c0 + t].ny;
  }
  for (int t = threadIdx.x; t < (c1 - c0) * nlayers; t += blockDim.x)
    s_T[t] = T[(size_t)c0 * nlayers + t];
  __syncthreads();
  if (i >= n) return;
  const double ax = fx[i], ay = fy[i];
  const int L = layer_of[i];
  double acc0 = 0.0, acc1 = 0.0;
  for (int c = 0; c < c1 - c0; ++c) {
    double th = s_nx[c] * ax + s_ny[c] * ay;
    th -= rint(th);
    double sn, cs;
    sincospi(2.0 * th, &sn, &cs);
    const double2 t = s_T[c * nlayers + L];
    acc0 += cs * t.x;
    acc1 += sn * t.y;
  }
  part[(size_t)chunk * n + i] = acc0 + acc1;
}

void launch_b_layer_project(hipStream_t st, int n, int ncols, int nlayers, const KCol* cols,
                            const int* layer_of, const double* layer_fz, const Buffers& b,
                            const double* sfw, double2* T, double* part) {
  hipLaunchKernelGGL(k_layer_sum, dim3(ncols), dim3(64), 0, st, ncols, nlayers, cols, layer_fz,
                     sfw, T);
  dim3 grid((n + 63) / 64, (ncols + LP_COLS - 1) / LP_COLS), block(64);
  hipLaunchKernelGGL(k_layer_project, grid, block, 0, st, n, ncols, nlayers, cols, layer_of,
                     b.efx, b.efy, T, part);
}

int layer_project_chunks(int ncols) { return (ncols + LP_COLS - 1) / LP_COLS; }

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
  __shared__ double s_zr[2][4];
  __shared__ int s_cnt[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int chunk = blockIdx.y;
  const int j0 = chunk * chunk_size, j1 = min(m, j0 + chunk_size);
  const double invLx = 1.0 / Lx, invLy = 1.0 / Ly, rc2 = rc * rc;
  const double r2_gauss = eta > alpha ? 45.0 / (eta * eta - alpha * alpha) : 1e300;
  const bool single = (Lx >= 2.0 * rc) && (Ly >= 2.0 * rc);
  double xi = 0, yi = 0, zi = 0;
  if (i < n) { xi = ex[i]; yi = ey[i]; zi = ez[i]; }
  // z interval of this workgroup's atoms: charges farther than rc from it
  // cannot contribute and are dropped when a tile is staged
  double zlo = i < n ? zi : 1e300, zhi = i < n ? zi : -1e300;
  for (int o = 32; o > 0; o >>= 1) {
    zlo = fmin(zlo, __shfl_xor(zlo, o, 64));
    zhi = fmax(zhi, __shfl_xor(zhi, o, 64));
  }
  if (lane == 0) { s_zr[0][wave] = zlo; s_zr[1][wave] = zhi; }
  __syncthreads();
  zlo = fmin(fmin(s_zr[0][0], s_zr[0][1]), fmin(s_zr[0][2], s_zr[0][3]));
  zhi = fmax(fmax(s_zr[1][0], s_zr[1][1]), fmax(s_zr[1][2], s_zr[1][3]));
  double acc = 0.0;
  for (int jt = j0; jt < j1; jt += RS_TILE) {
    const int nt = min(RS_TILE, j1 - jt);
    double x = 0, y = 0, z = 0, qq = 0;
    bool keep = false;
    if ((int)threadIdx.x < nt) {
      const int j = jt + threadIdx.x;
      x = xyz[3 * j]; y = xyz[3 * j + 1]; z = xyz[3 * j + 2];
      x -= Lx * floor(x * invLx);
      y -= Ly * floor(y * invLy);
      qq = q[j];
      keep = (z > zlo - rc) && (z < zhi + rc);
    }
    // order-preserving compaction: ballot within the wave, wave offsets via LDS
    const unsigned long long bal = __ballot(keep);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    __syncthreads();
    if (lane == 0) s_cnt[wave] = __popcll(bal);
    __syncthreads();
    int off = 0;
    for (int w2 = 0; w2 < wave; ++w2) off += s_cnt[w2];
    const int kept = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
    if (keep) {
      s_x[off + before] = x; s_y[off + before] = y; s_z[off + before] = z;
      s_q[off + before] = qq;
    }
    __syncthreads();
    if (i >= n) continue;
    for (int t = 0; t < kept; ++t) {
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

// b_i = -k_e (sum of k-space partials + sum of real-space partials
//            + (4 pi / V) z_i M_z), M_z from the structure-factor chunks.
// Four lanes per atom sum interleaved partial rows; the four sums are added
// in a fixed order.
__global__ void __launch_bounds__(256) k_combine(int n, int kchunks, int rchunks, int mchunks,
                                                 const double* __restrict__ phik,
                                                 const double* __restrict__ phir,
                                                 const double* __restrict__ ez,
                                                 const double* __restrict__ mz_part,
                                                 double slab_coef, double ke, void* out,
                                                 int out_is_f32) {
  __shared__ double sh[4][64];
  const int sub = threadIdx.x >> 6, li = threadIdx.x & 63;
  const int i = blockIdx.x * 64 + li;
  double acc = 0.0;
  if (i < n) {
    for (int c = sub; c < kchunks; c += 4) acc += phik[(size_t)c * n + i];
    for (int c = sub; c < rchunks; c += 4) acc += phir[(size_t)c * n + i];
  }
  sh[sub][li] = acc;
  __syncthreads();
  if (sub != 0 || i >= n) return;
  double mz = 0.0;
  for (int c = 0; c < mchunks; ++c) mz += mz_part[c];
  const double phi = (sh[0][li] + sh[1][li]) + (sh[2][li] + sh[3][li]);
  const double b = -ke * (phi + slab_coef * ez[i] * mz);
  if (out_is_f32)
    reinterpret_cast<float*>(out)[i] = (float)b;
  else
    reinterpret_cast<double*>(out)[i] = b;
}

void launch_b_combine(hipStream_t st, int n, int kchunks, int rchunks, int mchunks,
                      const double* phik, const double* phir, const Buffers& b,
                      const double* mz_part, double slab_coef, double ke, void* out,
                      int out_is_f32) {
  hipLaunchKernelGGL(k_combine, dim3((n + 63) / 64), dim3(256), 0, st, n, kchunks, rchunks,
                     mchunks, phik, phir, b.ez, mz_part, slab_coef, ke, out, out_is_f32);
}

}  // namespace cpm
