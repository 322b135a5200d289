// The electrolyte vector b, recomputed for every electrolyte configuration
// (Sec. II.A: the dominant cost of each step).  b is minus
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
#include <algorithm>
#include <cmath>
#include <cstring>

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
// part[(chunk * nk + k) * 2 + {0,1}] = partial S(k) over the chunk's charges.
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
                                                          int nzm, double* __restrict__ part) {
  extern __shared__ double2 tab[];                  // [tj][W]
  __shared__ double s_f[3][SF_TJ], s_q[SF_TJ];
  __shared__ double2 s_e1[3][SF_TJ];
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
}

int sf_tile(int nxm, int nym, int nzm) {
  const int W = nxm + nym + nzm + 3;
  int tj = (int)(30720 / (W * sizeof(double2)));   // <= 30 KB of dynamic LDS
  return tj < 1 ? 1 : (tj > SF_TJ ? SF_TJ : tj);
}

void launch_b_structure_factor(hipStream_t st, int fp32, int nruns, const KRun* runs, int nk, int m,
                               int mchunks, const double* xyz, const double* q, double Lx,
                               double Ly, double Lz, int nxm, int nym, int nzm, double* part) {
  const int chunk_size = (m + mchunks - 1) / mchunks;
  const int tj = sf_tile(nxm, nym, nzm);
  const size_t shm = (size_t)tj * (nxm + nym + nzm + 3) * sizeof(double2);
  dim3 grid((nruns + 255) / 256, mchunks), block(256);
  if (fp32)
    hipLaunchKernelGGL(k_structure_factor<float>, grid, block, shm, st, nruns, runs, nk, m,
                       chunk_size, tj, xyz, q, Lx, Ly, Lz, nxm, nym, nzm, part);
  else
    hipLaunchKernelGGL(k_structure_factor<double>, grid, block, shm, st, nruns, runs, nk, m,
                       chunk_size, tj, xyz, q, Lx, Ly, Lz, nxm, nym, nzm, part);
}

// ---------------------------------------------------------------------------
// Structure factors on FP64 matrix cores: per-charge phase tables, then one
// real GEMM per group of (k_x, k_y) columns (details at k_sf_mfma).
// ---------------------------------------------------------------------------
typedef double v4d_t __attribute__((ext_vector_type(4)));
constexpr int SFM_TJ = 16;             // charges per wave tile (4 MFMA k-steps)
constexpr int SFM_COLS = 16;           // columns per M tile (32 GEMM rows)

struct SfmWave {                        // wave-private LDS area
  double C[2 * SFM_COLS][SFM_TJ + 1];  // A operand rows (Re C, Im C) x charges
  double B[SFM_NB][16][SFM_TJ + 1];    // B operand per n block: columns (n, Re/Im) x charges
};

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double2 cmul2(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Dipole partials of one configuration for the 256 charges of this block
// (every thread of the block calls it): dip[d] = sum q_j r_jd in raw
// coordinates, the same sums in the same order as k_elyt_dipole.
__device__ inline void block_dipole(int m, int j, const double* __restrict__ xyz,
                                    const double* __restrict__ q, double* __restrict__ dip) {
  __shared__ double sh[3][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double v[3] = {0.0, 0.0, 0.0};
  if (j < m) {
    const double qq = q[j];
    v[0] = qq * xyz[3 * j]; v[1] = qq * xyz[3 * j + 1]; v[2] = qq * xyz[3 * j + 2];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    for (int o = 32; o > 0; o >>= 1) v[d] += __shfl_xor(v[d], o, 64);
    if (lane == 0) sh[d][wave] = v[d];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int d = threadIdx.x;
    dip[d] = (sh[d][0] + sh[d][1]) + (sh[d][2] + sh[d][3]);
  }
}

// Per-charge phase tables of one configuration, rows of mpad T2 entries
// (charges j >= m are zero):
//   rows [0, nxm]              X_a(j) = e^{2 pi i a fx_j}
//   rows nxm+1 + [0, 2 nym]    Y_b(j) = q_j e^{2 pi i (b - nym) fy_j}
//   next 8 rows                Z1_i(j) = e^{2 pi i i fz_j}
//   next nbz rows              Z8_c(j) = e^{2 pi i 8 c fz_j}
//   last row                   zero (the C operand of absent columns)
// One thread per (charge, row family, configuration) forms the family's
// entries as powers of its first phase in FP64 (complex products: a few
// 1e-15 relative after 30 powers), rounded once to T2 when stored.
// Families: X (n_x = 0..nxm), q Y (n_y = -nym..nym: powers and their
// conjugates), Z1 (n = 0..7), Z8 (8 n, n = 0..nbz-1) with the zero row.
// The X family's blocks also write the dipole partials of their 256 charges
// (blocks x 3 per configuration).  blockIdx.z selects the configuration of
// the group (tables tab_stride apart).
template <typename T2>
__global__ void __launch_bounds__(256) k_sf_tables(int m, int mpad, int nxm, int nym, int nbz,
                                                   const double* __restrict__ xyz,
                                                   const double* __restrict__ q, double Lx,
                                                   double Ly, double Lz, size_t tab_stride,
                                                   T2* __restrict__ tab, double* __restrict__ dip) {
  const int fam = blockIdx.y, snap = blockIdx.z;
  const int j = blockIdx.x * 256 + threadIdx.x;
  xyz += (size_t)snap * m * 3;
  if (fam == 0) block_dipole(m, j, xyz, q, dip + ((size_t)snap * gridDim.x + blockIdx.x) * 3);
  if (j >= mpad) return;
  const int rY = nxm + 1, rZ1 = rY + 2 * nym + 1, rZ8 = rZ1 + 8;
  tab += (size_t)snap * tab_stride + j;
  const bool live = j < m;
  double f = 0.0, scale = live ? 1.0 : 0.0;
  int row0 = 0, count = 0;
  double step = 1.0;                                 // power of the first phase per row
  if (fam == 0) {
    if (live) { f = xyz[3 * j] / Lx; f -= floor(f); }
    row0 = 0; count = nxm + 1;
  } else if (fam == 1) {
    if (live) { f = xyz[3 * j + 1] / Ly; f -= floor(f); scale = q[j]; }
    row0 = rY + nym; count = nym + 1;                // n_y = 0..nym here, conjugates below
  } else if (fam == 2) {
    if (live) { f = xyz[3 * j + 2] / Lz; f -= floor(f); }
    row0 = rZ1; count = 8;
  } else {
    if (live) { f = xyz[3 * j + 2] / Lz; f -= floor(f); }
    row0 = rZ8; count = nbz; step = 8.0;
    T2 zero;
    zero.x = 0.0; zero.y = 0.0;
    tab[(size_t)(rZ8 + nbz) * mpad] = zero;          // the zero row
  }
  double th = step * f;
  th -= rint(th);
  double sn, cs;
  sincospi(2.0 * th, &sn, &cs);
  double pr = scale, pi = 0.0;                       // scale * phase^0
  for (int k = 0; k < count; ++k) {
    T2 e;
    e.x = pr; e.y = pi;
    tab[(size_t)(row0 + k) * mpad] = e;
    if (fam == 1 && k > 0) {
      e.y = -pi;
      tab[(size_t)(row0 - k) * mpad] = e;
    }
    const double nr = pr * cs - pi * sn, ni = pr * sn + pi * cs;
    pr = nr;
    pi = ni;
  }
}

// ---------------------------------------------------------------------------
// The structure factors for b stored in FP32 on FP16 matrix cores with split
// operands.  Every operand value a (|a| <= max |q_j|) is carried as a pair of
// FP16 numbers, a_h = fp16(a) and a_l = fp16((a - a_h) 2^11) (the 2^11 keeps
// a_l in the normal FP16 range; below 2^-14 a_h may flush and a_l holds a),
// and a product of two values as
//   a b ~= a_h b_h + 2^-11 (a_h b_l + a_l b_h),
// three v_mfma_f32_16x16x32_f16 products into two FP32 accumulators.  Each
// value is kept to about 2^-22 relative (the dropped a_l b_l term is 2^-22 of
// the product), close to the FP32 rounding of the tables themselves.
//
// Tables of one configuration (float2 rows of mpad entries, then the z
// operand):
//   rows [0, nxm]                     X_a(j) = e^{2 pi i a fx_j}
//   rows nxm+1 + [0, 2 nym]           Y_b(j) = q_j e^{2 pi i (b - nym) fy_j}
//   next row                          zero (absent columns)
//   then nbz blocks of 8 mpad float2: the z operand of k_z block bb,
//     e^{2 pi i (8 bb + n) fz_j} (n = 0..7; column 2n + (0: Re, 1: Im)),
//     split into FP16 pairs, in matrix-core order: for charge group
//     jg = j / 8 and part h (0: a_h, 1: a_l) the 16 columns x 8 charges
//     at halfs ((bb (mpad / 8) + jg) 2 + h) 128 + 8 column + j % 8.
// ---------------------------------------------------------------------------
typedef _Float16 v8h_t __attribute__((ext_vector_type(8)));

int sf16_rows(int nxm, int nym, int nbz) { return (nxm + 1) + (2 * nym + 1) + 1 + 8 * nbz; }

constexpr int ZS_ROW = 264;              // halfs per LDS row of the z-operand staging
constexpr float SF16_LO = 2048.f;         // scale of the low FP16 part

// the pair of an FP64 value, formed from its FP32 rounding (2^-24 relative,
// below the 2^-22 of the pair); the clamp to the FP16 range (a no-op here)
// keeps the compiler from fusing the two roundings into one FP64 -> FP16
// conversion, which it would expand into integer code
__device__ inline void split_f16(double v, _Float16& h, _Float16& l) {
  const float vf = __builtin_amdgcn_fmed3f((float)v, -65504.f, 65504.f);
  h = (_Float16)vf;
  l = (_Float16)((vf - (float)h) * SF16_LO);
}

// grid (charge blocks of 256, 2 + nbz, configurations): y = 0 the X rows,
// the zero row and the dipole partials of the block's charges, y = 1 the Y
// rows, y = 2 + bb the z operand of block bb.  Phases are powers of a first
// one in FP64 (a few 1e-15 relative).
__global__ void __launch_bounds__(256) k_sf_tables16(int m, int mpad, int nxm, int nym, int nbz,
                                                     const double* __restrict__ xyz,
                                                     const double* __restrict__ q, double Lx,
                                                     double Ly, double Lz, size_t tab_stride,
                                                     float2* __restrict__ tab,
                                                     double* __restrict__ dip) {
  __shared__ __align__(16) _Float16 zs[32 * ZS_ROW];
  const int fam = blockIdx.y, snap = blockIdx.z;
  const int jb = blockIdx.x * 256, jl = threadIdx.x, j = jb + jl;
  const int rY = nxm + 1, rzero = rY + 2 * nym + 1;
  xyz += (size_t)snap * m * 3;
  tab += (size_t)snap * tab_stride;
  if (fam == 0) block_dipole(m, j, xyz, q, dip + ((size_t)snap * gridDim.x + blockIdx.x) * 3);
  const bool live = j < m;
  if (fam < 2) {
    if (j >= mpad) return;
    double f = 0.0, scale = live ? 1.0 : 0.0;
    int count;
    if (fam == 0) {
      if (live) { f = xyz[3 * j] / Lx; f -= floor(f); }
      count = nxm + 1;
      tab[(size_t)rzero * mpad + j] = make_float2(0.f, 0.f);
    } else {
      if (live) { f = xyz[3 * j + 1] / Ly; f -= floor(f); scale = q[j]; }
      count = nym + 1;
    }
    double sn, cs;
    sincospi(2.0 * f, &sn, &cs);
    double pr = scale, pi = 0.0;
    for (int k = 0; k < count; ++k) {
      if (fam == 0) {
        tab[(size_t)k * mpad + j] = make_float2((float)pr, (float)pi);
      } else {
        tab[(size_t)(rY + nym + k) * mpad + j] = make_float2((float)pr, (float)pi);
        if (k > 0) tab[(size_t)(rY + nym - k) * mpad + j] = make_float2((float)pr, (float)-pi);
      }
      const double nr = pr * cs - pi * sn, ni = pr * sn + pi * cs;
      pr = nr;
      pi = ni;
    }
    return;
  }
  // z operand of block bb = fam - 2: staged in LDS as 32 rows (part h,
  // column) of the block's 256 charges (rows ZS_ROW halfs apart, so the
  // 16-byte reads of the copy hit distinct banks), then stored as whole
  // 16-byte runs; every thread stays to the end (block barrier)
  const int bb = fam - 2;
  double f = 0.0;
  if (live) { f = xyz[3 * j + 2] / Lz; f -= floor(f); }
  double th = 8.0 * bb * f;
  th -= rint(th);
  double pr, pi, s1, c1;
  sincospi(2.0 * th, &pi, &pr);
  sincospi(2.0 * f, &s1, &c1);
  if (!live) { pr = 0.0; pi = 0.0; }
  for (int n = 0; n < 8; ++n) {
    _Float16 h, l;
    split_f16(pr, h, l);
    zs[(2 * n) * ZS_ROW + jl] = h;
    zs[(16 + 2 * n) * ZS_ROW + jl] = l;
    split_f16(pi, h, l);
    zs[(2 * n + 1) * ZS_ROW + jl] = h;
    zs[(16 + 2 * n + 1) * ZS_ROW + jl] = l;
    const double nr = pr * c1 - pi * s1, ni = pr * s1 + pi * c1;
    pr = nr;
    pi = ni;
  }
  __syncthreads();
  // block bb, charge groups jb/8 ..: per group 32 runs of 16 bytes (part h,
  // column), the runs of one group contiguous
  const int nvalid = min(256, mpad - jb);           // a multiple of 64
  uint4* dst = reinterpret_cast<uint4*>(tab + (size_t)(rzero + 1) * mpad) +
               ((size_t)bb * (mpad / 8) + jb / 8) * 32;
  for (int u = jl; u < nvalid * 4; u += 256)
    dst[u] = *reinterpret_cast<const uint4*>(zs + (u & 31) * ZS_ROW + (u >> 5) * 8);
}

int sf_table_rows(int nxm, int nym, int nbz) { return (nxm + 1) + (2 * nym + 1) + 8 + nbz + 1; }

void launch_b_sf_tables(hipStream_t st, int g, int m, int mpad, int nxm, int nym, int nbz,
                        const double* xyz, const double* q, double Lx, double Ly, double Lz,
                        double2* tab, int fp32, double* dip) {
  // blocks of 256 charges: as many as the dipole partials have (mpad is at
  // most the multiple of 256 above m)
  const int blocks = (mpad + 255) / 256;
  dim3 block(256);
  if (fp32 == 2) {
    hipLaunchKernelGGL(k_sf_tables16, dim3(blocks, 2 + nbz, g), block, 0, st, m, mpad, nxm, nym, nbz,
                       xyz, q, Lx, Ly, Lz, (size_t)sf16_rows(nxm, nym, nbz) * mpad,
                       reinterpret_cast<float2*>(tab), dip);
    return;
  }
  const size_t stride = (size_t)sf_table_rows(nxm, nym, nbz) * mpad;
  if (fp32)
    hipLaunchKernelGGL(k_sf_tables<float2>, dim3(blocks, 4, g), block, 0, st, m, mpad, nxm, nym, nbz,
                       xyz, q, Lx, Ly, Lz, stride, reinterpret_cast<float2*>(tab), dip);
  else
    hipLaunchKernelGGL(k_sf_tables<double2>, dim3(blocks, 4, g), block, 0, st, m, mpad, nxm, nym,
                       nbz, xyz, q, Lx, Ly, Lz, stride, tab, dip);
}

// Dipole partials of each configuration of a group, per 256 charges and
// axis: dip[((s * blocks + blk) * 3 + d] = sum q_j r_jd (raw coordinates; the
// dipole corrections of Eqs. 10-12 and 11 use them).  Positions and charges
// of configuration s start xyz_stride and q_stride elements apart (0: shared).
__global__ void __launch_bounds__(256) k_elyt_dipole(int m, const double* __restrict__ xyz,
                                                     size_t xyz_stride,
                                                     const double* __restrict__ q,
                                                     size_t q_stride, double* __restrict__ dip) {
  __shared__ double sh[3][4];
  const int j = blockIdx.x * 256 + threadIdx.x, snap = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double v[3] = {0.0, 0.0, 0.0};
  if (j < m) {
    const double* r = xyz + snap * xyz_stride + (size_t)j * 3;
    const double qq = q[snap * q_stride + j];
    v[0] = qq * r[0]; v[1] = qq * r[1]; v[2] = qq * r[2];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    for (int o = 32; o > 0; o >>= 1) v[d] += __shfl_xor(v[d], o, 64);
    if (lane == 0) sh[d][wave] = v[d];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int d = threadIdx.x;
    dip[((size_t)snap * gridDim.x + blockIdx.x) * 3 + d] = (sh[d][0] + sh[d][1]) + (sh[d][2] + sh[d][3]);
  }
}

void launch_b_elyt_dipole(hipStream_t st, int g, int m, const double* xyz, const double* q,
                          double* dip) {
  launch_dipole_partials(st, g, m, xyz, (size_t)m * 3, q, 0, dip);
}

void launch_dipole_partials(hipStream_t st, int g, int m, const double* xyz, size_t xyz_stride,
                            const double* q, size_t q_stride, double* dip) {
  hipLaunchKernelGGL(k_elyt_dipole, dim3((m + 255) / 256, g), dim3(256), 0, st, m, xyz, xyz_stride,
                     q, q_stride, dip);
}

// the electrolyte dipole of configuration s from its partials (fixed order)
__device__ inline void elyt_dipole(const double* __restrict__ dip, int blocks, int s, double M[3]) {
  M[0] = M[1] = M[2] = 0.0;
  for (int r = 0; r < blocks; ++r)
#pragma unroll
    for (int d = 0; d < 3; ++d) M[d] += dip[((size_t)s * blocks + r) * 3 + d];
}

// Structure factors of full (k_x, k_y) columns as a real GEMM on FP64 matrix
// cores.  For column c = (nx, ny) and charge j let C = q_j e^{i(kx x + ky y)}
// = X_nx(j) Y_ny(j) and Z = e^{i n kz1 z_j}; then over the charges
//   Pr = sum Re C Re Z,  Qr = sum Re C Im Z,  Pi = sum Im C Re Z,  Qi = sum Im C Im Z
// give S(c, +n) = (Pr - Qi) + i (Pi + Qr) and S(c, -n) = (Pr + Qi) + i (Pi - Qr)
// for n >= 0.  Columns are sorted by k_z extent and grouped 16 per M tile
// (32 rows); a work item is one M tile and at most SFM_NB blocks of 8
// consecutive n.  A workgroup takes one item and one chunk of charges; each
// wave walks its own tiles of 16 charges (no workgroup barrier inside the
// loop): it forms C from the X and Y tables and the first 8 phases of its n
// range from Z8 x Z1 into a wave-private LDS area, then runs
// v_mfma_f64_16x16x4f64 with the B operand advanced in registers by
// e^{2 pi i 8 fz} per 16-wide block.  The 4 waves are summed in a fixed order.
// Output, per configuration s and chunk: tile mt's 32 x 16 nb_mt block at
// part + (s * nchunks + chunk) * pchunk + toff[mt], row-major.
// The tile loop, the fixed-order wave sum and the store of one work item
// with NBW n blocks (NBW is uniform per workgroup: the kernel dispatches on
// it, so the per-block loops have no branches).  Per tile, each lane writes
// the B operand of its charge for two n of every block (e^{i n kz1 z},
// advanced by e^{2 pi i 8 fz} from block to block); the k steps then only
// read LDS and issue matrix-core products.
template <int NBW>
__device__ void sf_item(SfmWave& W, double* __restrict__ red, const double2* __restrict__ tab,
                        int mpad, int j0, int j1, const int (&xoff)[4], const int (&yoff)[4],
                        int z8off, int z1off, int r8off, double* __restrict__ out, int ldc,
                        int nb_lo) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int t_l = lane & 15, g_l = lane >> 4;
  v4d_t acc0[NBW], acc1[NBW];
#pragma unroll
  for (int b = 0; b < NBW; ++b) {
    acc0[b] = (v4d_t){0.0, 0.0, 0.0, 0.0};
    acc1[b] = (v4d_t){0.0, 0.0, 0.0, 0.0};
  }
  // table entries of the next tile are loaded while the current one runs
  double2 xv[4], yv[4], z8, za, zb, r8n;
  auto fetch = [&](int jt) {                        // jt + t_l < mpad: chunks are multiples of 16
#pragma unroll
    for (int u = 0; u < 4; ++u) { xv[u] = tab[xoff[u] + jt]; yv[u] = tab[yoff[u] + jt]; }
    z8 = tab[z8off + jt]; za = tab[z1off + jt]; zb = tab[z1off + mpad + jt]; r8n = tab[r8off + jt];
  };
  if (j0 + wave * SFM_TJ < j1) fetch(j0 + wave * SFM_TJ);
  for (int jt = j0 + wave * SFM_TJ; jt < j1; jt += 4 * SFM_TJ) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int cl = g_l + 4 * u;
      const double2 cv = cmul2(xv[u], yv[u]);
      W.C[2 * cl][t_l] = cv.x;
      W.C[2 * cl + 1][t_l] = cv.y;
    }
    // B columns 4 g_l .. 4 g_l + 3 (n = 2 g_l, 2 g_l + 1; Re, Im) of charge t_l
    double2 va = cmul2(z8, za), vb = cmul2(z8, zb);
#pragma unroll
    for (int b = 0; b < NBW; ++b) {
      W.B[b][4 * g_l][t_l] = va.x;
      W.B[b][4 * g_l + 1][t_l] = va.y;
      W.B[b][4 * g_l + 2][t_l] = vb.x;
      W.B[b][4 * g_l + 3][t_l] = vb.y;
      if (b + 1 < NBW) {
        va = cmul2(va, r8n);
        vb = cmul2(vb, r8n);
      }
    }
    wave_lds_sync();
    if (jt + 4 * SFM_TJ < j1) fetch(jt + 4 * SFM_TJ);
    // k step ks uses charges 4 ks + g_l of the tile
#pragma unroll 1
    for (int ks = 0; ks < SFM_TJ / 4; ++ks) {
      const int kc = 4 * ks + g_l;
      const double a0 = W.C[t_l][kc], a1 = W.C[16 + t_l][kc];
      double bv[NBW];
#pragma unroll
      for (int b = 0; b < NBW; ++b) bv[b] = W.B[b][t_l][kc];
#pragma unroll
      for (int b = 0; b < NBW; ++b) {
        acc0[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bv[b], acc0[b], 0, 0, 0);
        acc1[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv[b], acc1[b], 0, 0, 0);
      }
    }
    wave_lds_sync();
  }
  // fixed-order sum of the waves' accumulators (3 + 2 + 1 into wave 0)
  for (int src = 3; src >= 1; --src) {
    __syncthreads();
    if (wave == src)
#pragma unroll
      for (int b = 0; b < NBW; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          red[((0 * SFM_NB + b) * 4 + r) * 64 + lane] = acc0[b][r];
          red[((1 * SFM_NB + b) * 4 + r) * 64 + lane] = acc1[b][r];
        }
    __syncthreads();
    if (wave == 0)
#pragma unroll
      for (int b = 0; b < NBW; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          acc0[b][r] += red[((0 * SFM_NB + b) * 4 + r) * 64 + lane];
          acc1[b][r] += red[((1 * SFM_NB + b) * 4 + r) * 64 + lane];
        }
  }
  if (wave == 0) {
    // result register r of lane l: row (l >> 4) + 4 r, column l & 15 of block b
#pragma unroll
    for (int b = 0; b < NBW; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (lane >> 4) + 4 * r;
        const int col = 16 * (nb_lo + b) + (lane & 15);
        out[row * ldc + col] = acc0[b][r];
        out[(16 + row) * ldc + col] = acc1[b][r];
      }
  }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_sf_mfma(int mpad, int chunk_size, int nchunks, int nitems, const int4* __restrict__ items,
          const int* __restrict__ sc_nx, const int* __restrict__ sc_ny, int ncolsort, int nxm,
          int nym, const double2* __restrict__ tab, size_t tab_stride,
          const int* __restrict__ tile_nb, const int* __restrict__ toff, int pchunk,
          double* __restrict__ part) {
  // the waves' tile areas; after the tile loops, one wave's accumulators
  __shared__ double lds[4 * sizeof(SfmWave) / sizeof(double)];
  static_assert(64 * 2 * SFM_NB * 4 <= 4 * sizeof(SfmWave) / sizeof(double), "LDS reuse");
  SfmWave* wl = reinterpret_cast<SfmWave*>(lds);
  double* red = lds;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // workgroups go round-robin to the 8 XCDs; keep every (configuration,
  // charge chunk) pair on one XCD (pair = xcd mod 8) so its table rows stay
  // in that XCD's L2
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int item = slot % nitems;
  const int pair = xcd + 8 * (slot / nitems);
  const int snap = pair / nchunks, chunk = pair % nchunks;
  tab += (size_t)snap * tab_stride;
  const int4 it = items[item];
  const int mt = it.x, nb_lo = it.y, nbw = it.z;
  const int c_base = mt * SFM_COLS;
  const int ncol = min(SFM_COLS, ncolsort - c_base);
  const int j0 = chunk * chunk_size, j1 = min(mpad, j0 + chunk_size);
  const int t_l = lane & 15, g_l = lane >> 4;     // this lane's charge in the tile, lane group
  const int rY = nxm + 1, rZ1 = rY + 2 * nym + 1, rZ8 = rZ1 + 8;
  // table rows of this lane's four columns g_l + 4u (32-bit element offsets:
  // the tables stay far below 2^31 entries); columns past the end read the
  // zero row, so their C is zero
  const int rzero = (int)(tab_stride / mpad) - 1;
  int xoff[4], yoff[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int cl = g_l + 4 * u;
    const bool ok = cl < ncol;
    xoff[u] = (ok ? sc_nx[c_base + cl] : rzero) * mpad + t_l;
    yoff[u] = (ok ? rY + sc_ny[c_base + cl] + nym : rzero) * mpad + t_l;
  }
  const int z8off = (rZ8 + nb_lo) * mpad + t_l, r8off = (rZ8 + 1) * mpad + t_l;
  const int z1off = (rZ1 + 2 * g_l) * mpad + t_l;
  const int ldc = 16 * tile_nb[mt];
  double* out = part + ((size_t)snap * nchunks + chunk) * pchunk + toff[mt];
  SfmWave& W = wl[wave];
  switch (nbw) {
    case 1: sf_item<1>(W, red, tab, mpad, j0, j1, xoff, yoff, z8off, z1off, r8off, out, ldc, nb_lo); break;
    case 2: sf_item<2>(W, red, tab, mpad, j0, j1, xoff, yoff, z8off, z1off, r8off, out, ldc, nb_lo); break;
    case 3: sf_item<3>(W, red, tab, mpad, j0, j1, xoff, yoff, z8off, z1off, r8off, out, ldc, nb_lo); break;
    default: sf_item<SFM_NB>(W, red, tab, mpad, j0, j1, xoff, yoff, z8off, z1off, r8off, out, ldc, nb_lo); break;
  }
}

// The same structure factors on FP32 matrix cores, for b stored in FP32
// (the reduced-precision solve path): FP32 phase tables (each entry the FP64
// sincospi value rounded once), the C and B operands formed in FP32, and
// v_mfma_f32_16x16x4f32 products summed in FP32 over SF32_FLUSH tiles of a
// wave (128 charges), then added to FP64 accumulators, which the workgroup
// reduction and the partials keep.  The error this adds to b is a few 1e-7
// relative, below the rounding of b to FP32 itself.  Result register r of
// lane l: row 4 (l >> 4) + r, column l & 15.
typedef float v4f_t __attribute__((ext_vector_type(4)));
constexpr int SF32_FLUSH = 8;

struct SfmWave32 {                      // wave-private LDS area
  float C[2 * SFM_COLS][SFM_TJ + 1];
  float B[SFM_NB][16][SFM_TJ + 1];
};

__device__ inline float2 cmul2f(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int NBW>
__device__ void sf_item32(SfmWave32& W, double* __restrict__ red, const float2* __restrict__ tab,
                          int mpad, int j0, int j1, const int (&xoff)[4], const int (&yoff)[4],
                          int z8off, int z1off, int r8off, double* __restrict__ out, int ldc,
                          int nb_lo) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int t_l = lane & 15, g_l = lane >> 4;
  v4d_t acc0[NBW], acc1[NBW];
  v4f_t f0[NBW], f1[NBW];
#pragma unroll
  for (int b = 0; b < NBW; ++b) {
    acc0[b] = (v4d_t){0.0, 0.0, 0.0, 0.0};
    acc1[b] = (v4d_t){0.0, 0.0, 0.0, 0.0};
    f0[b] = (v4f_t){0.f, 0.f, 0.f, 0.f};
    f1[b] = (v4f_t){0.f, 0.f, 0.f, 0.f};
  }
  auto flush = [&]() {
#pragma unroll
    for (int b = 0; b < NBW; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc0[b][r] += (double)f0[b][r];
        acc1[b][r] += (double)f1[b][r];
      }
#pragma unroll
    for (int b = 0; b < NBW; ++b) {
      f0[b] = (v4f_t){0.f, 0.f, 0.f, 0.f};
      f1[b] = (v4f_t){0.f, 0.f, 0.f, 0.f};
    }
  };
  float2 xv[4], yv[4], z8, za, zb, r8n;
  auto fetch = [&](int jt) {
#pragma unroll
    for (int u = 0; u < 4; ++u) { xv[u] = tab[xoff[u] + jt]; yv[u] = tab[yoff[u] + jt]; }
    z8 = tab[z8off + jt]; za = tab[z1off + jt]; zb = tab[z1off + mpad + jt]; r8n = tab[r8off + jt];
  };
  if (j0 + wave * SFM_TJ < j1) fetch(j0 + wave * SFM_TJ);
  int since = 0;
  for (int jt = j0 + wave * SFM_TJ; jt < j1; jt += 4 * SFM_TJ) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int cl = g_l + 4 * u;
      const float2 cv = cmul2f(xv[u], yv[u]);
      W.C[2 * cl][t_l] = cv.x;
      W.C[2 * cl + 1][t_l] = cv.y;
    }
    float2 va = cmul2f(z8, za), vb = cmul2f(z8, zb);
#pragma unroll
    for (int b = 0; b < NBW; ++b) {
      W.B[b][4 * g_l][t_l] = va.x;
      W.B[b][4 * g_l + 1][t_l] = va.y;
      W.B[b][4 * g_l + 2][t_l] = vb.x;
      W.B[b][4 * g_l + 3][t_l] = vb.y;
      if (b + 1 < NBW) {
        va = cmul2f(va, r8n);
        vb = cmul2f(vb, r8n);
      }
    }
    wave_lds_sync();
    if (jt + 4 * SFM_TJ < j1) fetch(jt + 4 * SFM_TJ);
#pragma unroll 1
    for (int ks = 0; ks < SFM_TJ / 4; ++ks) {
      const int kc = 4 * ks + g_l;
      const float a0 = W.C[t_l][kc], a1 = W.C[16 + t_l][kc];
      float bv[NBW];
#pragma unroll
      for (int b = 0; b < NBW; ++b) bv[b] = W.B[b][t_l][kc];
#pragma unroll
      for (int b = 0; b < NBW; ++b) {
        f0[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, bv[b], f0[b], 0, 0, 0);
        f1[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, bv[b], f1[b], 0, 0, 0);
      }
    }
    wave_lds_sync();
    if (++since == SF32_FLUSH) {
      flush();
      since = 0;
    }
  }
  flush();
  // fixed-order sum of the waves' accumulators (3 + 2 + 1 into wave 0)
  for (int src = 3; src >= 1; --src) {
    __syncthreads();
    if (wave == src)
#pragma unroll
      for (int b = 0; b < NBW; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          red[((0 * SFM_NB + b) * 4 + r) * 64 + lane] = acc0[b][r];
          red[((1 * SFM_NB + b) * 4 + r) * 64 + lane] = acc1[b][r];
        }
    __syncthreads();
    if (wave == 0)
#pragma unroll
      for (int b = 0; b < NBW; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          acc0[b][r] += red[((0 * SFM_NB + b) * 4 + r) * 64 + lane];
          acc1[b][r] += red[((1 * SFM_NB + b) * 4 + r) * 64 + lane];
        }
  }
  if (wave == 0) {
#pragma unroll
    for (int b = 0; b < NBW; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 4 * (lane >> 4) + r;
        const int col = 16 * (nb_lo + b) + (lane & 15);
        out[row * ldc + col] = acc0[b][r];
        out[(16 + row) * ldc + col] = acc1[b][r];
      }
  }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_sf_mfma32(int mpad, int chunk_size, int nchunks, int nitems, const int4* __restrict__ items,
            const int* __restrict__ sc_nx, const int* __restrict__ sc_ny, int ncolsort, int nxm,
            int nym, const float2* __restrict__ tab, size_t tab_stride,
            const int* __restrict__ tile_nb, const int* __restrict__ toff, int pchunk,
            double* __restrict__ part) {
  // the waves' tile areas; after the tile loops, one wave's accumulators
  constexpr int LDS_D = (4 * sizeof(SfmWave32) + 7) / 8 > 64 * 2 * SFM_NB * 4
                            ? (4 * sizeof(SfmWave32) + 7) / 8 : 64 * 2 * SFM_NB * 4;
  __shared__ double lds[LDS_D];
  SfmWave32* wl = reinterpret_cast<SfmWave32*>(lds);
  double* red = lds;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int item = slot % nitems;
  const int pair = xcd + 8 * (slot / nitems);
  const int snap = pair / nchunks, chunk = pair % nchunks;
  tab += (size_t)snap * tab_stride;
  const int4 it = items[item];
  const int mt = it.x, nb_lo = it.y, nbw = it.z;
  const int c_base = mt * SFM_COLS;
  const int ncol = min(SFM_COLS, ncolsort - c_base);
  const int j0 = chunk * chunk_size, j1 = min(mpad, j0 + chunk_size);
  const int t_l = lane & 15, g_l = lane >> 4;
  const int rY = nxm + 1, rZ1 = rY + 2 * nym + 1, rZ8 = rZ1 + 8;
  const int rzero = (int)(tab_stride / mpad) - 1;
  int xoff[4], yoff[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int cl = g_l + 4 * u;
    const bool ok = cl < ncol;
    xoff[u] = (ok ? sc_nx[c_base + cl] : rzero) * mpad + t_l;
    yoff[u] = (ok ? rY + sc_ny[c_base + cl] + nym : rzero) * mpad + t_l;
  }
  const int z8off = (rZ8 + nb_lo) * mpad + t_l, r8off = (rZ8 + 1) * mpad + t_l;
  const int z1off = (rZ1 + 2 * g_l) * mpad + t_l;
  const int ldc = 16 * tile_nb[mt];
  double* out = part + ((size_t)snap * nchunks + chunk) * pchunk + toff[mt];
  SfmWave32& W = wl[wave];
  switch (nbw) {
    case 1: sf_item32<1>(W, red, tab, mpad, j0, j1, xoff, yoff, z8off, z1off, r8off, out, ldc, nb_lo); break;
    case 2: sf_item32<2>(W, red, tab, mpad, j0, j1, xoff, yoff, z8off, z1off, r8off, out, ldc, nb_lo); break;
    case 3: sf_item32<3>(W, red, tab, mpad, j0, j1, xoff, yoff, z8off, z1off, r8off, out, ldc, nb_lo); break;
    default: sf_item32<SFM_NB>(W, red, tab, mpad, j0, j1, xoff, yoff, z8off, z1off, r8off, out, ldc, nb_lo); break;
  }
}

// One work item (M tile of 16 columns, nbw <= SF16_NB blocks of 8 n) over
// one chunk of charges, in tiles of 32 charges (one matrix-core k step).  Per
// tile the four waves form the A operand together (wave w: charges 8w..8w+7,
// lane l: column l & 15 and two charges; Re C to row 2c, Im C to row 2c+1,
// split in FP32) into a double-buffered LDS area, one barrier, then each
// wave runs the products of its own blocks w, w + 4, w + 8 (the B operand
// read pre-split from the z operand, the next tile's entries in flight).
// Sums stay in FP32 over the chunk (at most a few thousand charges: tiles of
// 32 are summed inside the matrix core, the error grows as the square root
// of the tiles) and go to FP64 at the store.
constexpr int SF16_ROW = 40;             // halfs per LDS row of A (32 charges + pad)

// One wave's part: KW of the item's blocks (blk0 + 4k) for its NT M tiles
// (the B operand of a block serves them all); every wave forms its share of
// A and meets the one barrier per tile, whatever its KW.  Tiles go in pairs
// (chunks are multiples of 64 charges) with two register sets for the B
// operand, so each tile's loads are issued a tile ahead and no copy between
// the sets makes them complete early; the last pair loads itself again
// instead of testing.
template <int KW, int NT>
__device__ void sf_wave16(_Float16 (*As)[NT][2][32][SF16_ROW], const float2* __restrict__ tab,
                          const v8h_t* __restrict__ zop, int mpad, int j0, int j1,
                          const int (&xrow)[NT], const int (&yrow)[NT], double* const (&out)[NT],
                          const int (&ldc)[NT], const int (&nbt)[NT], int blk0) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i_l = lane & 15, g_l = lane >> 4;
  constexpr int K = KW > 0 ? KW : 1;
  v4f_t fh[NT][2][K], fl[NT][2][K];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        fh[t][rb][k] = (v4f_t){0.f, 0.f, 0.f, 0.f};
        fl[t][rb][k] = (v4f_t){0.f, 0.f, 0.f, 0.f};
      }
  // A share: column i_l of every M tile, charges c0, c0 + 1 of the tile
  const int c0 = 8 * wave + 2 * g_l;
  const float4* xp[NT];
  const float4* yp[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    xp[t] = reinterpret_cast<const float4*>(tab + xrow[t] + c0);
    yp[t] = reinterpret_cast<const float4*>(tab + yrow[t] + c0);
  }
  // B: block blk0 + 4k, charge group (jt >> 3) + g_l, column i_l (v8h units)
  const v8h_t* zp = zop + ((size_t)blk0 * (mpad / 8) + g_l) * 32 + i_l;
  const size_t zstep = (size_t)(mpad / 8) * 32 * 4;
  typedef _Float16 v2h_t __attribute__((ext_vector_type(2)));
  float4 xv[NT], yv[NT];
  auto load_a = [&](int jt) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      xv[t] = xp[t][jt / 2];
      yv[t] = yp[t][jt / 2];
    }
  };
  // A share of the tile whose operands are in xv, yv into LDS buffer buf
  auto form_a = [&](int buf) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const float4 x = xv[t], y = yv[t];
      const float r0 = x.x * y.x - x.y * y.y, i0 = x.x * y.y + x.y * y.x;
      const float r1 = x.z * y.z - x.w * y.w, i1 = x.z * y.w + x.w * y.z;
      const _Float16 hr0 = (_Float16)r0, hr1 = (_Float16)r1, hi0 = (_Float16)i0, hi1 = (_Float16)i1;
      *reinterpret_cast<v2h_t*>(&As[buf][t][0][2 * i_l][c0]) = (v2h_t){hr0, hr1};
      *reinterpret_cast<v2h_t*>(&As[buf][t][1][2 * i_l][c0]) =
          (v2h_t){(_Float16)((r0 - (float)hr0) * SF16_LO), (_Float16)((r1 - (float)hr1) * SF16_LO)};
      *reinterpret_cast<v2h_t*>(&As[buf][t][0][2 * i_l + 1][c0]) = (v2h_t){hi0, hi1};
      *reinterpret_cast<v2h_t*>(&As[buf][t][1][2 * i_l + 1][c0]) =
          (v2h_t){(_Float16)((i0 - (float)hi0) * SF16_LO), (_Float16)((i1 - (float)hi1) * SF16_LO)};
    }
  };
  auto load_b = [&](v8h_t (&bh)[K], v8h_t (&bl)[K], int jt) {
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      bh[k] = zp[k * zstep + (size_t)(jt >> 3) * 32];
      bl[k] = zp[k * zstep + (size_t)(jt >> 3) * 32 + 16];
    }
  };
  auto products = [&](int buf, const v8h_t (&bh)[K], const v8h_t (&bl)[K]) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const v8h_t ah = *reinterpret_cast<const v8h_t*>(&As[buf][t][0][16 * rb + i_l][8 * g_l]);
        const v8h_t al = *reinterpret_cast<const v8h_t*>(&As[buf][t][1][16 * rb + i_l][8 * g_l]);
#pragma unroll
        for (int k = 0; k < KW; ++k) {
          fh[t][rb][k] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[k], fh[t][rb][k], 0, 0, 0);
          fl[t][rb][k] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[k], fl[t][rb][k], 0, 0, 0);
          fl[t][rb][k] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[k], fl[t][rb][k], 0, 0, 0);
        }
      }
  };
  v8h_t b0h[K], b0l[K], b1h[K], b1l[K];
  load_a(j0);
  load_b(b0h, b0l, j0);
  for (int jt = j0; jt < j1; jt += 64) {
    // tile jt (buffer 0, set 0); tile jt + 32 loads ahead
    form_a(0);
    load_a(jt + 32);
    load_b(b1h, b1l, jt + 32);
    __syncthreads();
    if (KW > 0) products(0, b0h, b0l);
    // tile jt + 32 (buffer 1, set 1); the next pair's first tile loads ahead
    const int jn = min(jt + 64, j1 - 64);
    form_a(1);
    load_a(jn);
    load_b(b0h, b0l, jn);
    __syncthreads();
    if (KW > 0) products(1, b1h, b1l);
  }
  // result register r of lane l: row 4 (l >> 4) + r, column l & 15; a
  // tile's blocks past its own extent are dropped
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      if (blk0 + 4 * k >= nbt[t]) continue;
      const int col = 16 * (blk0 + 4 * k) + i_l;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          out[t][(16 * rb + 4 * g_l + r) * ldc[t] + col] =
              (double)fh[t][rb][k][r] + (double)fl[t][rb][k][r] / SF16_LO;
    }
}

// Items {M tile mt, first block, blocks, M tiles nt <= NT (mt .. mt + nt - 1)}.
template <int NT>
__device__ void sf_item16(const float2* __restrict__ tab, int mpad, int chunk_size, int nchunks,
                          int snap, int chunk, int4 it, const int* __restrict__ sc_nx,
                          const int* __restrict__ sc_ny, int ncolsort, int nxm, int nym,
                          const int* __restrict__ tile_nb, const int* __restrict__ toff,
                          int pchunk, double* __restrict__ part,
                          _Float16 (*As)[NT][2][32][SF16_ROW]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, i_l = lane & 15;
  const int mt = it.x, nb_lo = it.y, nbw = it.z, nt = it.w;
  const int rY = nxm + 1, rzero = rY + 2 * nym + 1;
  // chunk_size and mpad are multiples of 64: every tile pair lies inside [0, mpad)
  const int j0 = chunk * chunk_size, j1 = min(mpad, j0 + chunk_size);
  int xrow[NT], yrow[NT], ldc[NT], nbt[NT];
  double* out[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    // absent tiles and columns read the zero row; an absent tile stores nothing
    const bool tile = t < nt;
    const int c_base = (mt + t) * SFM_COLS;
    const bool ok = tile && i_l < min(SFM_COLS, ncolsort - c_base);
    xrow[t] = (ok ? sc_nx[c_base + i_l] : rzero) * mpad;
    yrow[t] = (ok ? rY + sc_ny[c_base + i_l] + nym : rzero) * mpad;
    ldc[t] = tile ? 16 * tile_nb[mt + t] : 0;
    nbt[t] = tile ? tile_nb[mt + t] : 0;
    out[t] = part + ((size_t)snap * nchunks + chunk) * pchunk + (tile ? toff[mt + t] : 0);
  }
  if (j0 >= j1) {
    // an empty chunk: zero partials of this item's blocks
    for (int t = 0; t < NT; ++t)
      for (int k = nb_lo + wave; k < min(nb_lo + nbw, nbt[t]); k += 4)
        for (int e = lane; e < 32 * 16; e += 64) out[t][(e >> 4) * ldc[t] + 16 * k + (e & 15)] = 0.0;
    return;
  }
  const v8h_t* zop = reinterpret_cast<const v8h_t*>(tab + (size_t)(rzero + 1) * mpad);
  // this wave's blocks: nb_lo + wave + 4k, k < kw (nbw <= SF16_NB = 12)
  const int kw = wave < nbw ? (nbw - wave + 3) / 4 : 0;
  const int blk0 = nb_lo + wave;
  // (items of four M tiles hold at most 8 blocks: kw <= 2)
  switch (kw) {
    case 0: sf_wave16<0, NT>(As, tab, zop, mpad, j0, j1, xrow, yrow, out, ldc, nbt, blk0); break;
    case 1: sf_wave16<1, NT>(As, tab, zop, mpad, j0, j1, xrow, yrow, out, ldc, nbt, blk0); break;
    case 2: sf_wave16<2, NT>(As, tab, zop, mpad, j0, j1, xrow, yrow, out, ldc, nbt, blk0); break;
    default: sf_wave16<(NT == 4 ? 2 : 3), NT>(As, tab, zop, mpad, j0, j1, xrow, yrow, out, ldc, nbt, blk0); break;
  }
}

template <int NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT == 1 ? 3 : 2)))
k_sf_mfma16(int mpad, int chunk_size, int nchunks, int nitems, const int4* __restrict__ items,
            const int* __restrict__ sc_nx, const int* __restrict__ sc_ny, int ncolsort, int nxm,
            int nym, const float2* __restrict__ tab, size_t tab_stride,
            const int* __restrict__ tile_nb, const int* __restrict__ toff, int pchunk,
            double* __restrict__ part) {
  __shared__ __align__(16) _Float16 As[2][NT][2][32][SF16_ROW];
  // (configuration, chunk) pairs stay on one XCD, as in the other kernels
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int item = slot % nitems;
  const int pair = xcd + 8 * (slot / nitems);
  const int snap = pair / nchunks, chunk = pair % nchunks;
  sf_item16<NT>(tab + (size_t)snap * tab_stride, mpad, chunk_size, nchunks, snap, chunk,
                items[item], sc_nx, sc_ny, ncolsort, nxm, nym, tile_nb, toff, pchunk, part, As);
}

void launch_b_sf_mfma(hipStream_t st, int g, int mpad, int nchunks, int nitems, const int4* items,
                      const int* sc_nx, const int* sc_ny, int ncolsort, int nxm, int nym, int nbz,
                      const double2* tab, const int* tile_nb, const int* toff, int pchunk,
                      double* part, int fp32, int sf16_nt) {
  // nchunks is a multiple of 8 (one residue class of pairs per XCD)
  const int chunk_size = sf_mfma_chunk(mpad, nchunks);
  const size_t tab_stride = (size_t)sf_table_rows(nxm, nym, nbz) * mpad;
  dim3 grid(nitems * nchunks * g), block(256);
  if (fp32 == 2) {
    // tile pairs of 64 charges: chunk bounds on multiples of 64 (mpad is one)
    const int chunk32 = ((mpad + nchunks - 1) / nchunks + 63) / 64 * 64;
    hipLaunchKernelGGL(sf16_nt == 4 ? k_sf_mfma16<4> : sf16_nt == 2 ? k_sf_mfma16<2> : k_sf_mfma16<1>,
                       grid, block, 0, st, mpad,
                       chunk32, nchunks, nitems, items, sc_nx, sc_ny, ncolsort, nxm, nym,
                       reinterpret_cast<const float2*>(tab), (size_t)sf16_rows(nxm, nym, nbz) * mpad,
                       tile_nb, toff, pchunk, part);
    return;
  }
  if (fp32) {
    hipLaunchKernelGGL(k_sf_mfma32, grid, block, 0, st, mpad, chunk_size, nchunks, nitems, items,
                       sc_nx, sc_ny, ncolsort, nxm, nym, reinterpret_cast<const float2*>(tab),
                       tab_stride, tile_nb, toff, pchunk, part);
    return;
  }
  hipLaunchKernelGGL(k_sf_mfma, grid, block, 0, st, mpad, chunk_size, nchunks, nitems, items, sc_nx,
                     sc_ny, ncolsort, nxm, nym, tab, tab_stride, tile_nb, toff, pchunk, part);
}

// Sum the chunks of the matrix-core structure factors and scatter them to
// the flat k order: thread per (sorted column, n >= 0); sfw = 2W S.
__global__ void k_sf_mfma_reduce(int ncolsort, int nchunks, int pchunk,
                                 const int* __restrict__ tile_nb, const int* __restrict__ toff,
                                 const int* __restrict__ sc_lo, const int* __restrict__ sc_len,
                                 const int* __restrict__ sc_koff, const double* __restrict__ part,
                                 const double* __restrict__ w2, double* __restrict__ sfw,
                                 const int* __restrict__ n_index) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_index[ncolsort]) return;
  // binary search of the column owning entry e
  int lo = 0, hi = ncolsort;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (n_index[mid] <= e) lo = mid; else hi = mid;
  }
  const int c = lo, n = e - n_index[c];
  const int mt = c / SFM_COLS, cl = c % SFM_COLS, ldc = 16 * tile_nb[mt];
  double pr = 0, qr = 0, pi = 0, qi = 0;
#pragma unroll 4
  for (int ch = 0; ch < nchunks; ++ch) {
    const double* base = part + (size_t)ch * pchunk + toff[mt];
    pr += base[(2 * cl) * ldc + 2 * n];
    qr += base[(2 * cl) * ldc + 2 * n + 1];
    pi += base[(2 * cl + 1) * ldc + 2 * n];
    qi += base[(2 * cl + 1) * ldc + 2 * n + 1];
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

void launch_b_sf_mfma_reduce(hipStream_t st, int ncolsort, int nchunks, int pchunk,
                             const int* tile_nb, const int* toff, const int* sc_lo,
                             const int* sc_len, const int* sc_koff, const int* n_index,
                             int n_total, const double* part, const double* w2, double* sfw) {
  hipLaunchKernelGGL(k_sf_mfma_reduce, dim3((n_total + 255) / 256), dim3(256), 0, st, ncolsort,
                     nchunks, pchunk, tile_nb, toff, sc_lo, sc_len, sc_koff, part, w2, sfw,
                     n_index);
}

// Planar electrodes: sum the chunks of the matrix-core structure factors and
// fold k_z into the electrode planes in one pass.  For sorted column c and
// plane L,
//   T(c, L) = sum_{n in column} 2W(c, n) S(c, n) e^{-i n kz1 z_L},
// so that phi_i = sum_c Re[e^{-i (kx x_i + ky y_i)} T(c, L_i)].  One workgroup
// per (column, configuration) with nw waves: wave w sums its own contiguous
// range of charge chunks (lanes take n >= 0), the nw partial sums are added in
// wave order, the weighted S(c, +-n) are kept in LDS, and the planes are
// spread over the waves (one fixed-order wave sum per plane).  nw follows the
// chunk count, so the summation order is fixed per launch shape.
// pz[L * nzt + n] = e^{-2 pi i n fz_L};  T is written as the real right-hand
// operand of the projection product: Tcat[(L M2 + 2c) 64 + s] = Re T(c, L),
// Tcat[(L M2 + 2c + 1) 64 + s] = Im T(c, L) for configuration s.
__global__ void __launch_bounds__(512) k_sf_layer_reduce(
    int ncolsort, int nchunks, int pchunk, int nlayers, int nzt, const int* __restrict__ tile_nb,
    const int* __restrict__ toff, const int* __restrict__ sc_lo, const int* __restrict__ sc_len,
    const int* __restrict__ sc_koff, const int* __restrict__ n_index,
    const double* __restrict__ part, const double* __restrict__ w2,
    const double2* __restrict__ pz, int M2, double* __restrict__ Tcat) {
  extern __shared__ double2 s_sw[];    // [2][ncnt]: S(+n) w, S(-n) w; then [nw][4][ncnt] sums
  const int c = blockIdx.x, snap = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int ncnt = n_index[c + 1] - n_index[c];        // n = 0 .. ncnt - 1
  double* s_red = reinterpret_cast<double*>(s_sw + 2 * ncnt);
  const int mt = c / SFM_COLS, cl = c % SFM_COLS, ldc = 16 * tile_nb[mt];
  const int clo = sc_lo[c], chi = sc_lo[c] + sc_len[c] - 1, koff = sc_koff[c];
  const double* base0 = part + (size_t)snap * nchunks * pchunk + toff[mt];
  const int c0 = wave * nchunks / nw, c1 = (wave + 1) * nchunks / nw;
  if (nw == 1 && ncnt <= 128) {
    // one wave: each lane keeps the weighted S(c, +-n) of its (at most two)
    // n in registers, so the chunk sums, the weights and the plane phases
    // are all in flight at once and no LDS is used; the same sums in the
    // same order as the general path below
    double2 sp[2], sm[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int n = lane + 64 * h;
      sp[h] = sm[h] = make_double2(0.0, 0.0);
      if (n >= ncnt) continue;
      double pr = 0, qr = 0, pi = 0, qi = 0;
#pragma unroll 4
      for (int ch = 0; ch < nchunks; ++ch) {
        const double* base = base0 + (size_t)ch * pchunk;
        pr += base[(2 * cl) * ldc + 2 * n];
        qr += base[(2 * cl) * ldc + 2 * n + 1];
        pi += base[(2 * cl + 1) * ldc + 2 * n];
        qi += base[(2 * cl + 1) * ldc + 2 * n + 1];
      }
      double tpr = 0, tqr = 0, tpi = 0, tqi = 0;
      tpr += pr;
      tqr += qr;
      tpi += pi;
      tqi += qi;
      if (n >= clo && n <= chi) {
        const double w = w2[koff + (n - clo)];
        sp[h] = make_double2(w * (tpr - tqi), w * (tpi + tqr));
      }
      if (n > 0 && -n >= clo && -n <= chi) {
        const double w = w2[koff + (-n - clo)];
        sm[h] = make_double2(w * (tpr + tqi), w * (tpi - tqr));
      }
    }
    for (int L = 0; L < nlayers; ++L) {
      double tr = 0.0, ti = 0.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int n = lane + 64 * h;
        if (n >= ncnt) continue;
        const double2 p = pz[(size_t)L * nzt + n];      // e^{-i n kz1 z_L}
        tr += (sp[h].x * p.x - sp[h].y * p.y) + (sm[h].x * p.x + sm[h].y * p.y);
        ti += (sp[h].x * p.y + sp[h].y * p.x) + (sm[h].y * p.x - sm[h].x * p.y);
      }
      for (int o = 32; o > 0; o >>= 1) {
        tr += __shfl_xor(tr, o, 64);
        ti += __shfl_xor(ti, o, 64);
      }
      if (lane == 0) {
        Tcat[((size_t)L * M2 + 2 * c) * 64 + snap] = tr;
        Tcat[((size_t)L * M2 + 2 * c + 1) * 64 + snap] = ti;
      }
    }
    return;
  }
  for (int n = lane; n < ncnt; n += 64) {
    double pr = 0, qr = 0, pi = 0, qi = 0;
#pragma unroll 4
    for (int ch = c0; ch < c1; ++ch) {
      const double* base = base0 + (size_t)ch * pchunk;
      pr += base[(2 * cl) * ldc + 2 * n];
      qr += base[(2 * cl) * ldc + 2 * n + 1];
      pi += base[(2 * cl + 1) * ldc + 2 * n];
      qi += base[(2 * cl + 1) * ldc + 2 * n + 1];
    }
    double* r = s_red + (size_t)wave * 4 * ncnt;
    r[n] = pr;
    r[ncnt + n] = qr;
    r[2 * ncnt + n] = pi;
    r[3 * ncnt + n] = qi;
  }
  __syncthreads();
  for (int n = threadIdx.x; n < ncnt; n += blockDim.x) {
    double pr = 0, qr = 0, pi = 0, qi = 0;
    for (int w = 0; w < nw; ++w) {
      const double* r = s_red + (size_t)w * 4 * ncnt;
      pr += r[n];
      qr += r[ncnt + n];
      pi += r[2 * ncnt + n];
      qi += r[3 * ncnt + n];
    }
    double2 sp = make_double2(0.0, 0.0), sm = make_double2(0.0, 0.0);
    if (n >= clo && n <= chi) {
      const double w = w2[koff + (n - clo)];
      sp = make_double2(w * (pr - qi), w * (pi + qr));
    }
    if (n > 0 && -n >= clo && -n <= chi) {
      const double w = w2[koff + (-n - clo)];
      sm = make_double2(w * (pr + qi), w * (pi - qr));
    }
    s_sw[n] = sp;
    s_sw[ncnt + n] = sm;
  }
  __syncthreads();
  for (int L = wave; L < nlayers; L += nw) {
    double tr = 0.0, ti = 0.0;
    for (int n = lane; n < ncnt; n += 64) {
      const double2 p = pz[(size_t)L * nzt + n];      // e^{-i n kz1 z_L}
      const double2 sp = s_sw[n], sm = s_sw[ncnt + n];
      // sp * p + sm * conj(p)
      tr += (sp.x * p.x - sp.y * p.y) + (sm.x * p.x + sm.y * p.y);
      ti += (sp.x * p.y + sp.y * p.x) + (sm.y * p.x - sm.x * p.y);
    }
    for (int o = 32; o > 0; o >>= 1) {
      tr += __shfl_xor(tr, o, 64);
      ti += __shfl_xor(ti, o, 64);
    }
    if (lane == 0) {
      Tcat[((size_t)L * M2 + 2 * c) * 64 + snap] = tr;
      Tcat[((size_t)L * M2 + 2 * c + 1) * 64 + snap] = ti;
    }
  }
}

void launch_b_sf_layer_reduce(hipStream_t st, int g, int ncolsort, int nchunks, int pchunk,
                              int nlayers, int nzt, int max_ncnt, const int* tile_nb,
                              const int* toff, const int* sc_lo, const int* sc_len,
                              const int* sc_koff, const int* n_index, const double* part,
                              const double* w2, const double2* pz, int M2, double* Tcat) {
  // about 8 chunks per wave, at most 8 waves, within 64 KB of LDS
  int nw = std::max(1, std::min(8, (nchunks + 7) / 8));
  auto lds = [&](int w) {
    return (size_t)2 * max_ncnt * sizeof(double2) + (size_t)w * 4 * max_ncnt * sizeof(double);
  };
  while (nw > 1 && lds(nw) > 65536) --nw;
  const size_t shm = lds(nw);
  hipLaunchKernelGGL(k_sf_layer_reduce, dim3(ncolsort, g), dim3(64 * nw), shm, st, ncolsort,
                     nchunks, pchunk, nlayers, nzt, tile_nb, toff, sc_lo, sc_len, sc_koff, n_index,
                     part, w2, pz, M2, Tcat);
}

// Plane phases pz[L * nzt + n] = e^{-2 pi i n fz_L}, fixed while the
// electrodes are.
__global__ void k_plane_phase(int nlayers, int nzt, const double* __restrict__ layer_fz,
                              double2* __restrict__ pz) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nlayers * nzt) return;
  const int L = e / nzt, nn = e % nzt;
  double th = nn * layer_fz[L];
  th -= rint(th);
  double sn, cs;
  sincospi(2.0 * th, &sn, &cs);
  pz[e] = make_double2(cs, -sn);
}

void launch_plane_phases(hipStream_t st, int nlayers, int nzt, const double* layer_fz,
                         double2* pz) {
  hipLaunchKernelGGL(k_plane_phase, dim3((nlayers * nzt + 255) / 256), dim3(256), 0, st, nlayers,
                     nzt, layer_fz, pz);
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

// Electrode-point pair function g(r) = (erfc(alpha r) - erfc(eta r)) / r
// (the Gaussian-smeared electrode charge seen from a point charge, minus
// the part carried by the Ewald k-space sum), tabulated on RS_NT equal
// intervals of [0, rc] as (g, g', g'') per node.  g is even and smooth at
// r = 0, so while eta r < 1.5 the nodes come from its Taylor series
// g = sum_k c_k r^{2k}, c_k = (2/sqrt(pi)) (-1)^k (eta^{2k+1} - alpha^{2k+1}) / (k! (2k+1));
// beyond, from h = erfc(alpha r) - erfc(eta r):  g = h/r, g' = (h' - g)/r,
// g'' = (h'' - 2 g')/r.  Quintic Hermite interpolation between the nodes
// reproduces g to a few 1e-15 (absolute, 1/A) at eta ~ 2, alpha ~ 0.3,
// rc ~ 12 A; the interpolation error grows as (eta rc / RS_NT)^6.
__global__ void k_pair_table(double alpha, double eta, double h, double* __restrict__ tab) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > RS_NT) return;
  const double r = k * h, two_rpi = 1.1283791670955126;   // 2 / sqrt(pi)
  double g, g1, g2;
  if (r * fmax(eta, alpha) < 1.5) {
    // Taylor series in r^2 while eta r < 1.5 (terms stay below ~2, so no
    // cancellation); 40 terms: the last is below 1e-33
    double a2k1 = alpha, e2k1 = eta, fact = 1.0, r2k = 1.0;
    const double a2 = alpha * alpha, e2 = eta * eta, r2 = r * r;
    g = 0.0; g1 = 0.0; g2 = 0.0;
    for (int kk = 0; kk < 40; ++kk) {
      const double ck = two_rpi * ((kk & 1) ? -1.0 : 1.0) * (e2k1 - a2k1) / (fact * (2 * kk + 1));
      g += ck * r2k;                                       // c_k r^{2k}
      if (kk >= 1 && k > 0) {
        g1 += 2.0 * kk * ck * r2k / r;                     // 2k c_k r^{2k-1}
        g2 += 2.0 * kk * (2.0 * kk - 1.0) * ck * r2k / r2; // 2k(2k-1) c_k r^{2k-2}
      }
      a2k1 *= a2; e2k1 *= e2; fact *= (kk + 1); r2k *= r2;
    }
    if (k == 0) { g1 = 0.0; g2 = 2.0 * (-two_rpi * (eta * e2 - alpha * a2) / 3.0); }
  } else {
    const double ea = exp(-alpha * alpha * r * r), ee = exp(-eta * eta * r * r);
    const double hv = erfc(alpha * r) - erfc(eta * r);
    const double h1 = two_rpi * (eta * ee - alpha * ea);
    const double h2 = 2.0 * two_rpi * r * (alpha * alpha * alpha * ea - eta * eta * eta * ee);
    g = hv / r;
    g1 = (h1 - g) / r;
    g2 = (h2 - 2.0 * g1) / r;
  }
  tab[3 * k] = g;
  tab[3 * k + 1] = g1;
  tab[3 * k + 2] = g2;
}

void launch_pair_table(hipStream_t st, double alpha, double eta, double rc, double* tab) {
  hipLaunchKernelGGL(k_pair_table, dim3((RS_NT + 1 + 255) / 256), dim3(256), 0, st, alpha, eta,
                     rc / RS_NT, tab);
}

// g(r) at r = sqrt(r2), 0 < r2 < rc^2, from the node table in LDS (quintic
// Hermite on the node's interval).  sqrt by the hardware reciprocal square
// root and two Newton steps (r2 is far from the denormal and overflow range
// here, so no rescaling is needed).
__device__ inline double pair_g(const double* __restrict__ T, double r2, double inv_h, double h) {
  r2 = fmax(r2, 1e-200);
  double y = __builtin_amdgcn_rsq(r2);
  double r = r2 * y, hy = 0.5 * y;
  double e = fma(-hy, r, 0.5);
  r = fma(r, e, r); hy = fma(hy, e, hy);
  e = fma(-r, r, r2);
  r = fma(e, hy, r);
  e = fma(-r, r, r2);
  r = fma(e, hy, r);
  const double u = r * inv_h;
  const int k = min((int)u, RS_NT - 1);
  const double t = u - k;
  const double* Tk = T + 3 * k;
  const double g0 = Tk[0], d0 = h * Tk[1], e0 = h * h * Tk[2];
  const double g1 = Tk[3], d1 = h * Tk[4], e1 = h * h * Tk[5];
  const double D = g1 - g0;
  const double c3 = 10.0 * D - 6.0 * d0 - 4.0 * d1 - 1.5 * e0 + 0.5 * e1;
  const double c4 = -15.0 * D + 8.0 * d0 + 7.0 * d1 + 1.5 * e0 - e1;
  const double c5 = 6.0 * D - 3.0 * d0 - 3.0 * d1 - 0.5 * e0 + 0.5 * e1;
  return g0 + t * (d0 + t * (0.5 * e0 + t * (c3 + t * (c4 + t * c5))));
}

// Order of the electrolyte charges for the real-space pass: a stable
// counting sort of configuration 0 by z (nbins equal bins of [0, Lz)), so
// that the 64-charge blocks of the gathered arrays are thin in z and most of
// them lie outside a given electrode plane's window.  One workgroup of
// ZS_WAVES waves; wave w owns the w-th contiguous segment of the charges:
// per-wave bin counts (LDS atomics), then each wave's first position in every
// bin (bins in order, and within a bin the segments in order), then every
// wave places its segment 64 charges at a time, ranking equal bins by
// ballots over the bin bits.  perm[pos] = j in ascending (bin, j); the order
// only affects which blocks a wave may skip and the (fixed) order of each
// atom's real-space sum.
constexpr int ZS_WAVES = 16;
constexpr int ZS_MAXBINS = 896;       // (ZS_WAVES + 1) x bins ints stay below 64 KB of LDS

__global__ void __launch_bounds__(64 * ZS_WAVES) k_zsort(int m, const double* __restrict__ xyz,
                                                         double Lz, int nbins, int nbits,
                                                         int* __restrict__ perm) {
  extern __shared__ int s_zs[];                        // [ZS_WAVES][nbins] counts; [nbins] totals
  int* tot = s_zs + ZS_WAVES * nbins;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int* mine = s_zs + wave * nbins;
  const double scale = nbins / Lz;
  auto bin = [&](int j) {
    const double z = xyz[3 * (size_t)j + 2];
    const double zw = z - Lz * floor(z / Lz);
    return min(nbins - 1, max(0, (int)(zw * scale)));
  };
  const int seg = (m + ZS_WAVES - 1) / ZS_WAVES;
  const int a = min(m, wave * seg), e = min(m, a + seg);
  for (int k = tid; k < ZS_WAVES * nbins; k += blockDim.x) s_zs[k] = 0;
  __syncthreads();
  for (int j = a + lane; j < e; j += 64) atomicAdd(&mine[bin(j)], 1);
  __syncthreads();
  for (int k = tid; k < nbins; k += blockDim.x) {
    int t = 0;
    for (int w = 0; w < ZS_WAVES; ++w) t += s_zs[w * nbins + k];
    tot[k] = t;
  }
  __syncthreads();
  if (wave == 0) {                                     // exclusive scan of the bin totals
    int running = 0;
    for (int k0 = 0; k0 < nbins; k0 += 64) {
      const int k = k0 + lane;
      const int c = k < nbins ? tot[k] : 0;
      int incl = c;
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
      }
      if (k < nbins) tot[k] = running + incl - c;
      running += __shfl(incl, 63, 64);
    }
  }
  __syncthreads();
  for (int k = tid; k < nbins; k += blockDim.x) {      // first position of each wave's run
    int p = tot[k];
    for (int w = 0; w < ZS_WAVES; ++w) {
      const int c = s_zs[w * nbins + k];
      s_zs[w * nbins + k] = p;
      p += c;
    }
  }
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int j0 = a; j0 < e; j0 += 64) {
    const int j = j0 + lane;
    const int key = j < e ? bin(j) : nbins;            // nbins: no charge
    unsigned long long same = ~0ull;
    for (int t = 0; t < nbits; ++t) {
      const bool bit = (key >> t) & 1;
      const unsigned long long bal = __ballot(bit);
      same &= bit ? bal : ~bal;
    }
    const int rank = __popcll(same & below);
    int pos = 0;
    if (key < nbins) pos = mine[key] + rank;
    wave_lds_sync();
    if (key < nbins) {
      if (pos < m) perm[pos] = j;
      if (rank == 0) mine[key] += __popcll(same);
    }
    wave_lds_sync();
  }
}

int zsort_bins(double Lz) {
  return std::max(1, std::min(ZS_MAXBINS, (int)std::ceil(Lz / 0.25)));
}

void launch_zsort(hipStream_t st, int m, const double* xyz, double Lz, int nbins, int* perm) {
  nbins = std::max(1, std::min(ZS_MAXBINS, nbins));
  int nbits = 1;
  while ((1 << nbits) <= nbins) ++nbits;
  hipLaunchKernelGGL(k_zsort, dim3(1), dim3(64 * ZS_WAVES), (size_t)(ZS_WAVES + 1) * nbins * sizeof(int),
                     st, m, xyz, Lz, nbins, nbits, perm);
}

// The charges of a launch group in the order perm (identity when null) as
// (x wrapped, y wrapped, z, q), rows of mpad64 entries per configuration,
// and the z range of each block of 64: zr[s * (mpad64 / 64) + blk].
__global__ void __launch_bounds__(64) k_gather_charges(int m, int mpad64,
                                                       const int* __restrict__ perm,
                                                       const double* __restrict__ xyz,
                                                       const double* __restrict__ q, double Lx,
                                                       double Ly, double4* __restrict__ cq,
                                                       double2* __restrict__ zr) {
  const int blk = blockIdx.x, s = blockIdx.y, lane = threadIdx.x;
  const int j = blk * 64 + lane;
  const double invLx = 1.0 / Lx, invLy = 1.0 / Ly;
  double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
  double zlo = 1e300, zhi = -1e300;
  if (j < m) {
    int src = perm ? perm[j] : j;
    if (src < 0 || src >= m) src = j;
    const double* r = xyz + ((size_t)s * m + src) * 3;
    const double x = r[0], y = r[1], z = r[2];
    v = make_double4(x - Lx * floor(x * invLx), y - Ly * floor(y * invLy), z, q[src]);
    zlo = zhi = z;
  }
  cq[(size_t)s * mpad64 + j] = v;
  for (int o = 32; o > 0; o >>= 1) {
    zlo = fmin(zlo, __shfl_xor(zlo, o, 64));
    zhi = fmax(zhi, __shfl_xor(zhi, o, 64));
  }
  if (lane == 0) zr[(size_t)s * (mpad64 / 64) + blk] = make_double2(zlo, zhi);
}

void launch_gather_charges(hipStream_t st, int g, int m, int mpad64, const int* perm,
                           const double* xyz, const double* q, double Lx, double Ly, double4* cq,
                           double2* zr) {
  hipLaunchKernelGGL(k_gather_charges, dim3(mpad64 / 64, g), dim3(64), 0, st, m, mpad64, perm, xyz,
                     q, Lx, Ly, cq, zr);
}

// Real-space part of phi_i over one chunk of the electrolyte, for the
// configurations s = blockIdx.z, blockIdx.z + gridDim.z, ... < g of a group
// (gathered charges cq and block z ranges zr of configuration s, rows mpad64
// and mpad64 / 64 apart; output rows part[(s * rchunks + chunk) * n + i]).
// Chunk c takes the 64-charge blocks c, c + rchunks, c + 2 rchunks, ... (so
// every chunk spans the whole z range of the ordered charges and the
// workgroups share the work evenly).  Threads map to electrode
// atoms through amap, which puts the atoms of one z plane, in compact
// in-plane tiles, into whole waves (-1 pads).  Every wave walks the chunk 64
// charges at a time on its own: a block whose z range misses the wave's z
// window is skipped without being loaded; otherwise the wave keeps the
// charges that can come within rc of its atoms -- the z window, and when
// every cell length is >= 2 rc (one image) an x and y window around the
// wave's atoms -- by order-preserving ballot compaction into a wave-private
// LDS area.  In the one-image case each lane then marks its possible
// partners in a 64-bit mask (an FP32 distance screen with a margin) and
// evaluates g(r) only for those within rc in FP64, in ascending order (the
// same pairs and order as a plain loop); otherwise it sums over all in-range
// images.  g(r) comes from the LDS pair table, staged once per workgroup of
// RS_WAVES waves.  The charges of the next three loaded blocks are in flight
// while the current one is summed.
constexpr int RS_WAVES = 8;

__global__ void __launch_bounds__(64 * RS_WAVES) k_real_space_b(
    int g, int n, int m, int mpad64, const int* __restrict__ amap, int nmap,
    const double* __restrict__ ex, const double* __restrict__ ey, const double* __restrict__ ez,
    const double4* __restrict__ cq, const double2* __restrict__ zr, double Lx, double Ly,
    double Lz, double rc, const double* __restrict__ ptab, double* __restrict__ part) {
  __shared__ double s_tab[3 * (RS_NT + 1)];
  __shared__ double s_c[RS_WAVES][4][64];              // per wave: x, y, z, q of kept charges
  __shared__ float s_cf[RS_WAVES][3][64];              // and x, y, z in FP32 for the screen
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  const int atom = slot < nmap ? amap[slot] : -1;
  const int chunk = blockIdx.y, rchunks = gridDim.y;
  const int nb64 = mpad64 / 64, nbt = (m + 63) / 64;   // blocks in a row, blocks holding charges
  const double invLx = 1.0 / Lx, invLy = 1.0 / Ly, invLz = 1.0 / Lz, rc2 = rc * rc;
  const double h = rc / RS_NT, inv_h = RS_NT / rc;
  // only the nearest image can lie within rc when every cell length is >= 2 rc
  const bool single = (Lx >= 2.0 * rc) && (Ly >= 2.0 * rc) && (Lz >= 2.0 * rc);
  for (int t = threadIdx.x; t < 3 * (RS_NT + 1); t += blockDim.x) s_tab[t] = ptab[t];
  __syncthreads();
  double xi = 0, yi = 0, zi = 0;
  if (atom >= 0) { xi = ex[atom]; yi = ey[atom]; zi = ez[atom]; }
  // this wave's extent in z (and x, y: wrapped coordinates)
  double zlo = atom >= 0 ? zi : 1e300, zhi = atom >= 0 ? zi : -1e300;
  double xlo = atom >= 0 ? xi : 1e300, xhi = atom >= 0 ? xi : -1e300;
  double ylo = atom >= 0 ? yi : 1e300, yhi = atom >= 0 ? yi : -1e300;
  for (int o = 32; o > 0; o >>= 1) {
    zlo = fmin(zlo, __shfl_xor(zlo, o, 64));
    zhi = fmax(zhi, __shfl_xor(zhi, o, 64));
    xlo = fmin(xlo, __shfl_xor(xlo, o, 64));
    xhi = fmax(xhi, __shfl_xor(xhi, o, 64));
    ylo = fmin(ylo, __shfl_xor(ylo, o, 64));
    yhi = fmax(yhi, __shfl_xor(yhi, o, 64));
  }
  // windows [lo - rc, hi + rc) of charges that can come within rc (some
  // periodic image of the charge must fall inside); x and y only with one image
  const double wlo = zlo - rc, whi = zhi + rc;
  const bool keep_all_z = whi - wlo >= Lz;
  const double xw = xhi - xlo + 2.0 * rc, yw = yhi - ylo + 2.0 * rc;
  const bool keep_all_x = !single || xw >= Lx, keep_all_y = !single || yw >= Ly;
  double (*C)[64] = s_c[wave];
  float (*Cf)[64] = s_cf[wave];
  // FP32 screen of partners within rc: r2 in FP32 against rc^2 (1 + 1e-4),
  // which exceeds its rounding error for coordinates up to ~1e3 A, then the
  // exact FP64 test on the marked pairs
  const float xif = (float)xi, yif = (float)yi, zif = (float)zi;
  const float Lxf = (float)Lx, Lyf = (float)Ly, Lzf = (float)Lz;
  const float iLxf = 1.0f / Lxf, iLyf = 1.0f / Lyf, iLzf = 1.0f / Lzf;
  const float rc2f = (float)(rc2 * (1.0 + 1e-4));
  const int nblk = chunk < nbt ? (nbt - chunk + rchunks - 1) / rchunks : 0;
  const int s0 = blockIdx.z, sstep = gridDim.z;
  const int nloc = s0 < g ? (g - s0 + sstep - 1) / sstep : 0;   // this workgroup's configurations
  const int steps = nloc * nblk;
  // a block can hold a charge of the window when its z range, moved into
  // [wlo, wlo + Lz), starts below whi or wraps past wlo + Lz (a margin of
  // 1e-9 A keeps the test conservative under rounding); wave-uniform
  auto hit = [&](int step) {
    if (step >= steps) return false;
    if (keep_all_z) return true;
    const int snap = s0 + sstep * (step / nblk), gb = chunk + rchunks * (step % nblk);
    const double2 r = zr[(size_t)snap * nb64 + gb];
    const double a = r.x - Lz * floor((r.x - wlo) * invLz), w = r.y - r.x;
    return a < whi + 1e-9 || a + w >= wlo + Lz - 1e-9;
  };
  auto fetch = [&](int step, bool h) {
    double4 v = make_double4(0, 0, 0, 0);
    if (h) {                                           // h: step < steps, so nblk > 0
      const int snap = s0 + sstep * (step / nblk);
      const int j = (chunk + rchunks * (step % nblk)) * 64 + lane;
      if (j < m) v = cq[(size_t)snap * mpad64 + j];
    }
    return v;
  };
  bool h0 = hit(0), h1 = hit(1), h2 = hit(2);
  double4 f0 = fetch(0, h0), f1 = fetch(1, h1), f2 = fetch(2, h2);
  double acc = 0.0;
  for (int step = 0; step < steps; ++step) {
    const int snap = s0 + sstep * (step / nblk), blk = step % nblk;
    const bool hcur = h0;
    const double xw0 = f0.x, yw0 = f0.y, z = f0.z, qq = f0.w;
    f0 = f1;
    f1 = f2;
    h0 = h1;
    h1 = h2;
    h2 = hit(step + 3);
    f2 = fetch(step + 3, h2);
    if (hcur) {
      const bool valid = (chunk + rchunks * blk) * 64 + lane < m;
      bool keep = valid && (keep_all_z || (z - Lz * floor((z - wlo) * invLz)) < whi);
      if (!keep_all_x) {
        double d = xw0 - (xlo - rc);
        d -= Lx * floor(d * invLx);
        keep = keep && d < xw;
      }
      if (!keep_all_y) {
        double d = yw0 - (ylo - rc);
        d -= Ly * floor(d * invLy);
        keep = keep && d < yw;
      }
      const unsigned long long bal = __ballot(keep);
      const int kept = __popcll(bal);
      if (keep) {
        const int pos = __popcll(bal & ((1ull << lane) - 1ull));
        C[0][pos] = xw0;
        C[1][pos] = yw0;
        C[2][pos] = z;
        C[3][pos] = qq;
        Cf[0][pos] = (float)xw0;
        Cf[1][pos] = (float)yw0;
        Cf[2][pos] = (float)z;
      }
      wave_lds_sync();
      if (atom >= 0) {
        if (single) {
          // partners within rc (FP32 screen), then the exact test and g(r)
          // for those only, in ascending t
          unsigned long long mask = 0ull;
          for (int t = 0; t < kept; ++t) {
            float dz = zif - Cf[2][t], dx = xif - Cf[0][t], dy = yif - Cf[1][t];
            dz -= Lzf * rintf(dz * iLzf);
            dx -= Lxf * rintf(dx * iLxf);
            dy -= Lyf * rintf(dy * iLyf);
            if (dx * dx + dy * dy + dz * dz < rc2f) mask |= 1ull << t;
          }
          while (mask) {
            const int t = __ffsll((long long)mask) - 1;
            mask &= mask - 1ull;
            double dz = zi - C[2][t], dx = xi - C[0][t], dy = yi - C[1][t];
            dz -= Lz * rint(dz * invLz);
            dx -= Lx * rint(dx * invLx);
            dy -= Ly * rint(dy * invLy);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rc2) acc += C[3][t] * pair_g(s_tab, r2, inv_h, h);
          }
        } else {
          for (int t = 0; t < kept; ++t) {
            double dz = zi - C[2][t];
            dz -= Lz * rint(dz * invLz);
            if (fabs(dz) >= rc) continue;          // dz is the nearest image
            double dx = xi - C[0][t], dy = yi - C[1][t];
            dx -= Lx * rint(dx * invLx);
            dy -= Ly * rint(dy * invLy);
            const int alo = (int)ceil((-rc - dx) * invLx) - 1, ahi = (int)floor((rc - dx) * invLx) + 1;
            const int blo = (int)ceil((-rc - dy) * invLy) - 1, bhi = (int)floor((rc - dy) * invLy) + 1;
            const int clo = (int)ceil((-rc - dz) * invLz) - 1, chi = (int)floor((rc - dz) * invLz) + 1;
            for (int cc = clo; cc <= chi; ++cc) {
              const double Z = dz + cc * Lz;
              for (int a = alo; a <= ahi; ++a) {
                const double X = dx + a * Lx;
                for (int bb = blo; bb <= bhi; ++bb) {
                  const double Y = dy + bb * Ly;
                  const double r2 = X * X + Y * Y + Z * Z;
                  if (r2 < rc2) acc += C[3][t] * pair_g(s_tab, r2, inv_h, h);
                }
              }
            }
          }
        }
      }
      wave_lds_sync();
    }
    if (blk == nblk - 1) {
      if (atom >= 0) part[((size_t)snap * rchunks + chunk) * n + atom] = acc;
      acc = 0.0;
    }
  }
  if (nblk == 0 && atom >= 0)
    for (int snap = s0; snap < g; snap += sstep) part[((size_t)snap * rchunks + chunk) * n + atom] = 0.0;
}

// ---------------------------------------------------------------------------
// Real-space pair sum for electrodes on z planes when one periodic image at
// most lies within rc (every cell length >= 2 rc).
//
// g(r) = (erfc(alpha r) - erfc(eta r)) / r as a polynomial in s = r^2 on each
// of RP_N intervals of [0, rc] (uniform in r): degree RP_DEG in
// (s - s_mid), interpolated at the Chebyshev nodes of the interval, so no
// square root is taken in FP64 (an FP32 one picks the interval; a neighbouring
// interval's polynomial is as accurate just past its ends).  Absolute error a
// few 1e-14 against g(0) ~ 2 (alpha 0.18 .. 0.3, eta 1.979, rc = 3.6 / alpha).
// ---------------------------------------------------------------------------
namespace {
double pair_g_host(double r, double alpha, double eta) {
  const double two_rpi = 1.1283791670955126;   // 2 / sqrt(pi)
  if (r * std::max(alpha, eta) < 1.5) {
    // Taylor series in r^2 (no cancellation while eta r < 1.5)
    double a2k1 = alpha, e2k1 = eta, fact = 1.0, r2k = 1.0, g = 0.0;
    const double a2 = alpha * alpha, e2 = eta * eta, r2 = r * r;
    for (int k = 0; k < 40; ++k) {
      g += two_rpi * ((k & 1) ? -1.0 : 1.0) * (e2k1 - a2k1) / (fact * (2 * k + 1)) * r2k;
      a2k1 *= a2; e2k1 *= e2; fact *= (k + 1); r2k *= r2;
    }
    return g;
  }
  return (std::erfc(alpha * r) - std::erfc(eta * r)) / r;
}
}  // namespace

void pair_poly_table(double alpha, double eta, double rc, std::vector<double>& tab) {
  constexpr int D = RP_DEG;
  tab.assign((size_t)RP_N * RP_REC, 0.0);
  const double h = rc / RP_N, pi = 3.14159265358979323846;
  double node[D + 1];
  for (int i = 0; i <= D; ++i) node[i] = std::cos((2 * i + 1) * pi / (2.0 * (D + 1)));
  // monomial coefficients of the Chebyshev polynomials T_0 .. T_D
  double T[D + 1][D + 1] = {};
  T[0][0] = 1.0;
  T[1][1] = 1.0;
  for (int j = 2; j <= D; ++j)
    for (int p = 0; p <= D; ++p)
      T[j][p] = (p > 0 ? 2.0 * T[j - 1][p - 1] : 0.0) - T[j - 2][p];
  for (int k = 0; k < RP_N; ++k) {
    // s in [(k h)^2, ((k + 1) h)^2] = s_mid + hw [-1, 1]
    const double smid = h * h * ((double)k * (k + 1) + 0.5), hw = h * h * (k + 0.5);
    double f[D + 1], c[D + 1], b[D + 1] = {};
    for (int i = 0; i <= D; ++i) f[i] = pair_g_host(std::sqrt(smid + hw * node[i]), alpha, eta);
    for (int j = 0; j <= D; ++j) {
      double acc = 0.0;
      for (int i = 0; i <= D; ++i) acc += f[i] * std::cos(j * (2 * i + 1) * pi / (2.0 * (D + 1)));
      c[j] = acc * (j == 0 ? 1.0 : 2.0) / (D + 1);
    }
    for (int j = 0; j <= D; ++j)
      for (int p = 0; p <= D; ++p) b[p] += c[j] * T[j][p];
    // coefficients of (s - s_mid)^p: p <= 3 in FP64, p >= 4 in FP32 (those
    // terms stay below 2e-7 of g, so FP32 adds < 1e-14 of g); 48 bytes per
    // interval, so the intervals of a wave's lanes spread over the LDS banks
    double a[D + 1];
    double scale = 1.0;
    for (int p = 0; p <= D; ++p) {
      a[p] = b[p] / scale;
      scale *= hw;
    }
    double* rec = tab.data() + (size_t)k * RP_REC;
    for (int p = 0; p < 4; ++p) rec[p] = a[p];
    const float hi[4] = {(float)a[4], (float)a[5], (float)a[6], 0.0f};
    std::memcpy(rec + 4, hi, sizeof hi);
  }
}

// One wave per 64 atom-map slots of one z plane (slot tiles are compact in
// x and y).  The charges of a chunk arrive 64 at a time (z-sorted blocks; a
// block whose z range misses [z_p - rc, z_p + rc] is skipped unread).  A
// charge within rc of the plane in z is taken relative to the tile centre,
// in each image (x, y shifted by at most one cell length) that can come
// within rc of the tile's bounding box, and appended to the wave's ring of
// 128 entries:
//   FP32  (-2 dx, -2 dy) and W = dx^2 + dy^2 - (rc^2 - dz^2) - margin, so that
//         an atom at (ax, ay) from the centre is within rc when
//         ax (-2 dx) + ay (-2 dy) + W < -(ax^2 + ay^2)  (screen, margin
//         above its rounding error);
//   FP64  (dx, dy, dz^2, q) for the exact test and g.
// Every 64 entries each lane screens them into a 64-bit mask and evaluates
// the marked ones in FP64 (s < rc^2 exactly).  Two images of one charge are
// 2 rc or more apart, so an atom meets at most one of them within rc.  The
// summation order of an atom is fixed by the data (deterministic).
constexpr int RP_RING = 128;
struct RpWave {
  float2 c[RP_RING];
  float w[RP_RING];
  double4 d[RP_RING];
};

__global__ void __launch_bounds__(64 * RS_WAVES, 4) k_real_space_plane(
    int g, int n, int m, int mpad64, const int* __restrict__ amap, int nmap,
    const double* __restrict__ ex, const double* __restrict__ ey, const double* __restrict__ ez,
    const double4* __restrict__ cq, const double2* __restrict__ zr, double Lx, double Ly,
    double Lz, double rc, const double* __restrict__ ptab, double* __restrict__ part) {
  __shared__ __align__(16) double s_tab[RP_N * RP_REC];
  __shared__ RpWave s_w[RS_WAVES];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  const int atom = slot < nmap ? amap[slot] : -1;
  const int chunk = blockIdx.y, rchunks = gridDim.y;
  const int nb64 = mpad64 / 64, nbt = (m + 63) / 64;
  for (int t = threadIdx.x; t < RP_N * RP_REC / 2; t += blockDim.x)
    reinterpret_cast<double2*>(s_tab)[t] = reinterpret_cast<const double2*>(ptab)[t];
  __syncthreads();
  const unsigned long long valid_atoms = __ballot(atom >= 0);
  if (!valid_atoms) return;                      // a wave of padding slots only
  const double invLx = 1.0 / Lx, invLy = 1.0 / Ly, invLz = 1.0 / Lz, rc2 = rc * rc;
  double xi = 0, yi = 0, zi = 0;
  if (atom >= 0) { xi = ex[atom]; yi = ey[atom]; zi = ez[atom]; }
  xi -= Lx * floor(xi * invLx);
  yi -= Ly * floor(yi * invLy);
  // the plane's z (every atom of the wave shares it) and the tile's box
  const int first = __ffsll((long long)valid_atoms) - 1;
  const double zp = __shfl(zi, first, 64);
  double xlo = atom >= 0 ? xi : 1e300, xhi = atom >= 0 ? xi : -1e300;
  double ylo = atom >= 0 ? yi : 1e300, yhi = atom >= 0 ? yi : -1e300;
  for (int o = 32; o > 0; o >>= 1) {
    xlo = fmin(xlo, __shfl_xor(xlo, o, 64));
    xhi = fmax(xhi, __shfl_xor(xhi, o, 64));
    ylo = fmin(ylo, __shfl_xor(ylo, o, 64));
    yhi = fmax(yhi, __shfl_xor(yhi, o, 64));
  }
  const double cx = 0.5 * (xlo + xhi), cy = 0.5 * (ylo + yhi);
  const double hx = 0.5 * (xhi - xlo), hy = 0.5 * (yhi - ylo);
  const double ax = xi - cx, ay = yi - cy;
  const float axf = (float)ax, ayf = (float)ay, nAf = -(float)(ax * ax + ay * ay);
  // FP32 screen margin: its rounding error is below 50 u M^2 (u = 2^-24,
  // M the largest coordinate magnitude, rc + the tile's half extent)
  const double M = rc + fmax(hx, hy);
  const double marg = 4e-6 * M * M;
  RpWave& W = s_w[wave];
  const float inv_hf = (float)(RP_N / rc);
  const double hh = (rc / RP_N) * (rc / RP_N);   // s_mid of interval k: hh (k (k + 1) + 1/2)
  const int nblk = chunk < nbt ? (nbt - chunk + rchunks - 1) / rchunks : 0;
  const int s0 = blockIdx.z, sstep = gridDim.z;
  const int nloc = s0 < g ? (g - s0 + sstep - 1) / sstep : 0;
  const double wlo = zp - rc, whi = zp + rc;
  // does block blk of configuration snap reach the plane's z window?
  auto hit = [&](int snap, int blk) {
    const double2 r = zr[(size_t)snap * nb64 + chunk + rchunks * blk];
    const double a = r.x - Lz * floor((r.x - wlo) * invLz), w = r.y - r.x;
    return a < whi + 1e-9 || a + w >= wlo + Lz - 1e-9;
  };
  auto fetch = [&](int snap, int blk) {
    double4 v = make_double4(0, 0, 0, 0);
    if (blk >= 0) {
      const int j = (chunk + rchunks * blk) * 64 + lane;
      if (j < m) v = cq[(size_t)snap * mpad64 + j];
    }
    return v;
  };
  // screen entries [base, base + len) of the ring and add the marked pairs
  double acc = 0.0;
  auto process = [&](int base, int len) {
    if (atom >= 0) {
      unsigned long long mk = 0ull;
#pragma unroll 1
      for (int q4 = 0; q4 < 64; q4 += 16) {
        unsigned int mq = 0u;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const float2 c = W.c[base + q4 + t];
          const float v = fmaf(axf, c.x, fmaf(ayf, c.y, W.w[base + q4 + t]));
          mq |= (v < nAf) ? (1u << t) : 0u;
        }
        mk |= (unsigned long long)mq << q4;
      }
      if (len < 64) mk &= (1ull << len) - 1ull;
      while (mk) {
        const int t = __builtin_ctzll(mk);
        mk &= mk - 1ull;
        const double4 e = W.d[base + t];
        const double rx = ax - e.x, ry = ay - e.y;
        const double sv = fma(rx, rx, fma(ry, ry, e.z));
        const float rf = __builtin_amdgcn_sqrtf((float)sv);   // picks the interval only
        const int k = min((int)(rf * inv_hf), RP_N - 1);
        const double* T = s_tab + k * RP_REC;
        const double2 c01 = *reinterpret_cast<const double2*>(T);
        const double2 c23 = *reinterpret_cast<const double2*>(T + 2);
        const float4 c46 = *reinterpret_cast<const float4*>(T + 4);
        const double x = sv - hh * ((double)k * (double)(k + 1) + 0.5);   // s - s_mid
        const float xf = (float)x;
        const float th = fmaf(fmaf(c46.z, xf, c46.y), xf, c46.x);       // a6 x^2 + a5 x + a4
        double p = fma((double)th, x, c23.y);
        p = fma(p, x, c23.x);
        p = fma(p, x, c01.y);
        p = fma(p, x, c01.x);
        acc = fma(sv < rc2 ? e.w : 0.0, p, acc);
      }
    }
    wave_lds_sync();                             // the ring's entries are reused next
  };
  // per configuration: the blocks that reach the window, found 64 at a time
  // (one z-range load per lane, no load waits on another), then taken in
  // order with the charges of the next two in flight
  int head = 0, tail = 0;                        // ring window [head, tail), head in {0, 64}
  for (int li = 0; li < nloc; ++li) {
    const int snap = s0 + sstep * li;
    for (int b0 = 0; b0 < nblk; b0 += 64) {
      unsigned long long hm = __ballot(b0 + lane < nblk && hit(snap, b0 + lane));
      auto pop = [&]() {
        if (!hm) return -1;
        const int t = __builtin_ctzll(hm);
        hm &= hm - 1ull;
        return b0 + t;
      };
      int bA = pop(), bB = pop();
      double4 fA = fetch(snap, bA), fB = fetch(snap, bB);
      while (bA >= 0) {
        const int blk = bA;
        const double4 cur = fA;
        bA = bB;
        fA = fB;
        bB = pop();
        fB = fetch(snap, bB);
        const bool valid = (chunk + rchunks * blk) * 64 + lane < m;
        double dz = cur.z - zp;
        dz -= Lz * rint(dz * invLz);
        const double rho2 = rc2 - dz * dz;
        double dx = cur.x - cx, dy = cur.y - cy;
        dx -= Lx * rint(dx * invLx);
        dy -= Ly * rint(dy * invLy);
        const double dx2 = dx - copysign(Lx, dx), dy2 = dy - copysign(Ly, dy);
        // images whose distance from the tile's box can be below sqrt(rho2)
        auto near = [&](double px, double py) {
          const double ux = fmax(fabs(px) - hx, 0.0), uy = fmax(fabs(py) - hy, 0.0);
          return ux * ux + uy * uy < rho2 + marg;
        };
        int cand = 0;
        if (valid && fabs(dz) < rc) {
          cand = (near(dx, dy) ? 1 : 0) | (near(dx2, dy) ? 2 : 0) | (near(dx, dy2) ? 4 : 0) |
                 (near(dx2, dy2) ? 8 : 0);
        }
        while (true) {
          const bool has = cand != 0;
          const unsigned long long bal = __ballot(has);
          if (!bal) break;
          if (has) {
            const int which = __builtin_ctz(cand);
            cand &= cand - 1;
            const double px = (which & 1) ? dx2 : dx, py = (which & 2) ? dy2 : dy;
            const int pos = (tail + __popcll(bal & ((1ull << lane) - 1ull))) & (RP_RING - 1);
            W.c[pos] = make_float2((float)(-2.0 * px), (float)(-2.0 * py));
            W.w[pos] = (float)(px * px + py * py - rho2 - marg);
            W.d[pos] = make_double4(px, py, dz * dz, cur.w);
          }
          tail += __popcll(bal);
          wave_lds_sync();
          if (tail - head >= 64) {
            process(head & (RP_RING - 1), 64);
            head += 64;
          }
        }
      }
    }
    if (tail > head) process(head & (RP_RING - 1), tail - head);
    head = tail = 0;
    if (atom >= 0) part[((size_t)snap * rchunks + chunk) * n + atom] = acc;
    acc = 0.0;
  }
}

void launch_b_real_space(hipStream_t st, int g, int n, int m, int mpad64, int rchunks,
                         const Buffers& b, int nmap, const double4* cq, const double2* zr,
                         double Lx, double Ly, double Lz, double rc, double* part, int wg_target,
                         const double* plane_tab) {
  // configurations spread over the third grid dimension, about wg_target
  // workgroups in all (a workgroup loops over the configurations beyond)
  const int ablk = (nmap + 64 * RS_WAVES - 1) / (64 * RS_WAVES);
  const int gz = std::max(1, std::min(g, (wg_target + ablk * rchunks - 1) / (ablk * rchunks)));
  dim3 grid(ablk, rchunks, gz), block(64 * RS_WAVES);
  if (plane_tab)
    hipLaunchKernelGGL(k_real_space_plane, grid, block, 0, st, g, n, m, mpad64, b.amap, nmap,
                       b.ex, b.ey, b.ez, cq, zr, Lx, Ly, Lz, rc, plane_tab, part);
  else
    hipLaunchKernelGGL(k_real_space_b, grid, block, 0, st, g, n, m, mpad64, b.amap, nmap,
                       b.ex, b.ey, b.ez, cq, zr, Lx, Ly, Lz, rc, b.rtab, part);
}

// b_i = -k_e (sum of k-space partials + sum of real-space partials
//            + sum_d c_d r_id M_d): the electrolyte part of the geometry's
// dipole term (slab: c_z = 4 pi / V, Eq. 12; wire: c_x = c_y = 2 pi / V,
// Eq. 11; tin foil: none), M from the electrolyte dipole partials.
// Four lanes per atom sum interleaved partial rows; the four sums are added
// in a fixed order.
__global__ void __launch_bounds__(256) k_combine(int n, int kchunks, int rchunks,
                                                 const double* __restrict__ phik,
                                                 const double* __restrict__ phir,
                                                 const double* __restrict__ ex,
                                                 const double* __restrict__ ey,
                                                 const double* __restrict__ ez,
                                                 const double* __restrict__ dip, int dip_blocks,
                                                 double cx, double cy, double cz, double ke,
                                                 void* out, int out_is_f32) {
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
  double M[3];
  elyt_dipole(dip, dip_blocks, 0, M);
  const double phi = (sh[0][li] + sh[1][li]) + (sh[2][li] + sh[3][li]);
  const double b = -ke * (phi + (cx * ex[i] * M[0] + cy * ey[i] * M[1] + cz * ez[i] * M[2]));
  if (out_is_f32)
    reinterpret_cast<float*>(out)[i] = (float)b;
  else
    reinterpret_cast<double*>(out)[i] = b;
}

// Planar electrodes, a group of g configurations: b_i = -k_e (k-space
// potential + sum of real-space partials + sum_d c_d r_id M_d).  A workgroup
// takes 64 atoms of one configuration s with four lanes per atom; lane group
// u sums the parts q = u, u + 4, ... and the real-space chunks k = u, u + 4,
// ..., and the four sums are added in a fixed order.  The k-space parts of
// atom i are the rows the projection product left in its slot:
// Phi[(q nslot + slot_of[i]) 64 + s].
__global__ void __launch_bounds__(256) k_b_final(int n, int nslot, int nparts,
                                                 const int* __restrict__ slot_of,
                                                 const double* __restrict__ Phi,
                                                 const double* __restrict__ phir, int rchunks,
                                                 const double* __restrict__ ex,
                                                 const double* __restrict__ ey,
                                                 const double* __restrict__ ez,
                                                 const double* __restrict__ dip, int dip_blocks,
                                                 double cx, double cy, double cz, double ke,
                                                 void* out, int out_is_f32) {
  __shared__ double sh[4][64];
  const int sub = threadIdx.x >> 6, li = threadIdx.x & 63, s = blockIdx.y;
  const int i = blockIdx.x * 64 + li;
  double acc = 0.0;
  if (i < n) {
    const size_t r = slot_of[i];
    for (int q = sub; q < nparts; q += 4) acc += Phi[((size_t)q * nslot + r) * 64 + s];
#pragma unroll 4
    for (int k = sub; k < rchunks; k += 4) acc += phir[((size_t)s * rchunks + k) * n + i];
  }
  sh[sub][li] = acc;
  __syncthreads();
  if (sub != 0 || i >= n) return;
  double M[3];
  elyt_dipole(dip, dip_blocks, s, M);
  const double phi = (sh[0][li] + sh[1][li]) + (sh[2][li] + sh[3][li]);
  const double bv = -ke * (phi + (cx * ex[i] * M[0] + cy * ey[i] * M[1] + cz * ez[i] * M[2]));
  if (out_is_f32)
    reinterpret_cast<float*>(out)[(size_t)s * n + i] = (float)bv;
  else
    reinterpret_cast<double*>(out)[(size_t)s * n + i] = bv;
}

void launch_b_final(hipStream_t st, int g, int n, int nslot, int nparts, const int* slot_of,
                    const double* Phi, const double* phir, int rchunks, const Buffers& b,
                    const double* dip, int dip_blocks, const double* cdip, double ke, void* out,
                    int out_is_f32) {
  hipLaunchKernelGGL(k_b_final, dim3((n + 63) / 64, g), dim3(256), 0, st, n, nslot, nparts,
                     slot_of, Phi, phir, rchunks, b.ex, b.ey, b.ez, dip, dip_blocks, cdip[0],
                     cdip[1], cdip[2], ke, out, out_is_f32);
}

int real_space_block_atoms() { return 64 * RS_WAVES; }

void launch_b_combine(hipStream_t st, int n, int kchunks, int rchunks, const double* phik,
                      const double* phir, const Buffers& b, const double* dip, int dip_blocks,
                      const double* cdip, double ke, void* out, int out_is_f32) {
  hipLaunchKernelGGL(k_combine, dim3((n + 63) / 64), dim3(256), 0, st, n, kchunks, rchunks, phik,
                     phir, b.ex, b.ey, b.ez, dip, dip_blocks, cdip[0], cdip[1], cdip[2], ke, out,
                     out_is_f32);
}

}  // namespace cpm
