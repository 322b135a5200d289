// Matrix-free elastance operator and the projected conjugate-gradient solve.
//
// The charges minimise the electrostatic energy under charge neutrality
// (Sec. II.A; the conjugate-gradient route it names as the alternative to
// inverting A): q solves A q = b + v + mu e with e^T q = 0.  Conjugate
// gradients on the neutral subspace (projector P = I - e e^T / n) need only
// products A p, never A^-1 or S:
//   * real space + Gaussian self term: a fixed sparse matrix (every pair with
//     some periodic image within r_c), evaluated with the same expression as
//     the dense assembly, first as ELL rows and then kept as dense 64 x 64
//     blocks of the slot tiles that interact (the atoms of a plane are
//     ordered in compact 64-atom tiles), applied as FP64 matrix-core products
//     fused with the k-space projection;
//   * k space for electrodes on z planes: with E_j(c) = e^{i (kx x_j + ky y_j)}
//     and Q_c(L, L') = sum_n 2W(c, n) e^{i n kz1 (z_L - z_L')},
//       (A_k p)_i = k_e sum_c Re[conj(E_i(c)) T(c, L_i)],
//       T(c, L) = sum_L' Q_c(L', L) Y(c, L'),  Y(c, L') = sum_{j in L'} E_j(c) p_j,
//     the planar regrouping of A's k-space term applied to vectors: Y and the
//     projection are FP64 matrix-core products (K = the atoms of a plane, and
//     K = 2 x columns), T a small per-column mixing of the planes;
//   * background -pi/(V alpha^2) (sum p) and the geometry's dipole term
//     sum_d c_d r_id (sum_j r_jd p_j) from four moments of p;
//   * the optional per-atom diagonal.
//
// Layout: vectors are slot-major, V[slot * 64 + s] for up to 64 right-hand
// sides s, slots in the order of the atom map (the atoms of each z plane fill
// whole 64-slot tiles, -1 pads; for the dense A, slots are the atoms in
// caller order padded to a multiple of 64).  A wave owns one slot row at a
// time, lane s its vector s, so per-vector sums need no cross-lane
// reductions.  Every reduction runs in a fixed order and without
// inter-block communication inside a kernel: each block writes partials, and
// every block of the next kernel adds them in the same order (so all derive
// identical CG scalars).
#include <algorithm>

#include "cpm_internal.h"

namespace cpm {

namespace {

constexpr int VL = CG_MAXG;        // vectors per slot row
constexpr int CG_WAVES = 16;       // waves per block of the vector kernels
constexpr int CG_BLK = 64 * CG_WAVES;

// per-vector scalars for the host, scal[row * VL + s] (written by block 0)
enum { S_RR = 0, S_RR0, S_ITERS };
// block partial fields, red[(blk * CG_RED + f) * VL + s]; r.r alternates
// between two fields by iteration parity, and so does r.z of the
// preconditioned iteration (F_RZ, F_RZ + 1; producers: the preconditioner's
// tile blocks)
enum { F_PAP = 0, F_SAP, F_RR, F_RRB, F_RRI, F_SUM, F_M0, F_RZ = F_M0 + 4, F_RZB, F_ZSUM };
static_assert(F_ZSUM < CG_RED, "partial fields");
static_assert(S_ITERS < CG_NSCAL, "scalar rows");

// this wave's rows: r = (blk + t nblk) * CG_WAVES + wave, t = 0, 1, ...
struct Rows {
  int r, step;
  __device__ Rows() {
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    r = blockIdx.x * CG_WAVES + w;
    step = CG_WAVES * gridDim.x;
  }
};

// sum of 16 wave values per lane, sh[w][s] (w = 0..15), as a fixed tree
__device__ inline double sum16(const double (*sh)[VL], int s) {
  double a[8];
#pragma unroll
  for (int w = 0; w < 8; ++w) a[w] = sh[2 * w][s] + sh[2 * w + 1][s];
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// add the 16 waves' per-lane values v[0..NF) of this block and store them as
// block partials of fields f[0..NF) (threads 0..63)
template <int NF>
__device__ void store_partials(const double (&v)[NF], const int (&f)[NF],
                               double* __restrict__ red) {
  __shared__ double sh[NF][CG_WAVES][VL];
  const int s = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NF; ++k) sh[k][w][s] = v[k];
  __syncthreads();
  if (threadIdx.x < VL) {
#pragma unroll
    for (int k = 0; k < NF; ++k) red[((size_t)blockIdx.x * CG_RED + f[k]) * VL + s] = sum16(sh[k], s);
  }
}

// Totals over the nprod blocks of the producing kernel of fields f[0..NF),
// computed by every block of the consuming kernel in the same fixed order
// (wave w adds blocks w, w + 16, ..., then a fixed tree over the waves), so
// all blocks see identical values without any inter-block communication.
// out[k][s] is valid for all threads after the call.
template <int NF>
__device__ void block_totals(const double* __restrict__ red, int nprod, const int (&f)[NF],
                             double (*out)[VL]) {
  __shared__ double sh[NF][CG_WAVES][VL];
  const int s = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    double a = 0.0;
    for (int b = w; b < nprod; b += CG_WAVES) a += red[((size_t)b * CG_RED + f[k]) * VL + s];
    sh[k][w][s] = a;
  }
  __syncthreads();
  if (threadIdx.x < VL) {
#pragma unroll
    for (int k = 0; k < NF; ++k) out[k][s] = sum16(sh[k], s);
  }
  __syncthreads();
}

// ---- real-space + self part of A in ELL form (slot space) -----------------
// The periodic-image sum of one electrode pair, written as in the dense
// assembly: every image with 0 < r < r_c, erfc(eta_ee r) dropped once it is
// below FP64 rounding of the difference.  Returns the number of images
// within range.
__device__ inline int pair_images(double dx, double dy, double dz, double Lx, double Ly,
                                  double Lz, double rc, double alpha, double eta_ee,
                                  double* sum) {
  const double invLx = 1.0 / Lx, invLy = 1.0 / Ly, invLz = 1.0 / Lz, rc2 = rc * rc;
  const double r2_gauss = eta_ee > alpha ? 45.0 / (eta_ee * eta_ee - alpha * alpha) : 1e300;
  dx -= Lx * rint(dx * invLx);
  dy -= Ly * rint(dy * invLy);
  dz -= Lz * rint(dz * invLz);
  int cnt = 0;
  double acc = 0.0;
  if (fabs(dz) < rc) {
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
          if (r2 > 0.0 && r2 < rc2 * (1.0 + 1e-12)) {
            const double r = sqrt(r2);
            if (r < rc) {
              acc += (r2 > r2_gauss ? erfc(alpha * r) : erfc(alpha * r) - erfc(eta_ee * r)) / r;
              ++cnt;
            }
          }
        }
      }
    }
  }
  *sum = acc;
  return cnt;
}

// One pass over the slot chunk of row r.  FILL = false counts the entries
// (cnt[chunk nslot + r]); FILL = true writes them (row-major, r * width + k)
// from offset cnt[chunk nslot + r] on, never past kend (the next chunk's
// offset, or the width for the last chunk).  Both passes run this same code,
// so they take the same in-range decisions.
template <bool FILL>
__global__ void __launch_bounds__(256) k_ell_pass(int nslot, int chunk, int width,
                                                  const int* __restrict__ slot_atom,
                                                  const double* __restrict__ ex,
                                                  const double* __restrict__ ey,
                                                  const double* __restrict__ ez, double Lx,
                                                  double Ly, double Lz, double rc, double alpha,
                                                  double eta_ee, double diag_self,
                                                  int* __restrict__ cnt, int* __restrict__ col,
                                                  double* __restrict__ val) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, ch = blockIdx.y;
  if (r >= nslot) return;
  const int i = slot_atom[r];
  size_t k = FILL ? (size_t)cnt[(size_t)ch * nslot + r] : 0;
  const size_t kend = FILL ? (ch + 1 < (int)gridDim.y ? (size_t)cnt[(size_t)(ch + 1) * nslot + r]
                                                      : (size_t)width)
                           : 0;
  if (i >= 0) {
    const int j0 = ch * chunk, j1 = min(nslot, j0 + chunk);
    const double xi = ex[i], yi = ey[i], zi = ez[i];
    for (int t = j0; t < j1; ++t) {
      const int j = slot_atom[t];
      if (j < 0) continue;
      double s;
      const int c = pair_images(xi - ex[j], yi - ey[j], zi - ez[j], Lx, Ly, Lz, rc, alpha, eta_ee, &s);
      if (j == i || c > 0) {
        if (FILL && k < kend) {
          col[(size_t)r * width + k] = t;
          val[(size_t)r * width + k] = (j == i) ? s + diag_self : s;
        }
        ++k;
      }
    }
  }
  if (!FILL) cnt[(size_t)ch * nslot + r] = (int)k;
}

// padding entries: column = own slot, value 0
__global__ void k_ell_init(int width, size_t total, int* __restrict__ col,
                           double* __restrict__ val) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  col[e] = (int)(e / width);
  val[e] = 0.0;
}

// In-plane phases in slot order as a real matrix: Ecat[(2c) nslot + slot] =
// cos th, Ecat[(2c + 1) nslot + slot] = sin th, th = kx x + ky y of column c;
// zero for pad slots and for padding columns c >= ncolsort.
__global__ void k_cg_ephase(int nslot, int ncolsort, const int* __restrict__ slot_atom,
                            const int* __restrict__ sc_nx, const int* __restrict__ sc_ny,
                            const double* __restrict__ fx, const double* __restrict__ fy,
                            double* __restrict__ Ecat) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (r >= nslot) return;
  const int i = slot_atom[r];
  double cs = 0.0, sn = 0.0;
  if (i >= 0 && c < ncolsort) {
    double th = sc_nx[c] * fx[i] + sc_ny[c] * fy[i];
    th -= rint(th);
    sincospi(2.0 * th, &sn, &cs);
  }
  Ecat[(size_t)(2 * c) * nslot + r] = cs;
  Ecat[(size_t)(2 * c + 1) * nslot + r] = sn;
}

// ---- k space and real space on matrix cores ---------------------------------
// 64 x 64 output tiles (64 slot or column rows m, 64 vectors s) per 256-thread
// workgroup: 4 waves in 2 x 2 quadrants of 2 x 2 v_mfma_f64_16x16x4f64
// blocks, K staged through LDS in slabs of 16 with the next slab held in
// registers.  MFMA operand layout (lane l): A (row l % 16, k l / 16), B
// (k l / 16, col l % 16); result register q: (row l / 16 + 4 q, col l % 16).
typedef double v4d __attribute__((ext_vector_type(4)));

// acc += A (64 x K) B (K x 64) for one segment, K a multiple of 16.
// A(m, k) = A[m lda + k] (ACOL = false) or A[k lda + m] (ACOL = true);
// B(k, s) = B[k VL + s].
template <bool ACOL>
__device__ void seg_mfma(v4d (&acc)[2][2], const double* __restrict__ A, size_t lda,
                         const double* __restrict__ B, int K, double (*As)[68],
                         double (*Bs)[68]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  double ra[4], rb[4];
  auto load = [&](int k0) {
    if (!ACOL) {
      const int r = tid >> 2, c = (tid & 3) * 4;
      const double* src = A + (size_t)r * lda + k0 + c;
      for (int t = 0; t < 4; ++t) ra[t] = src[t];
    } else {
      const int r = tid >> 4, c = (tid & 15) * 4;
      const double* src = A + (size_t)(k0 + r) * lda + c;
      for (int t = 0; t < 4; ++t) ra[t] = src[t];
    }
    const int r = tid >> 4, c = (tid & 15) * 4;
    const double* src = B + (size_t)(k0 + r) * VL + c;
    for (int t = 0; t < 4; ++t) rb[t] = src[t];
  };
  auto store = [&]() {
    if (!ACOL) {
      const int r = tid >> 2, c = (tid & 3) * 4;
      for (int t = 0; t < 4; ++t) As[c + t][r] = ra[t];
    } else {
      const int r = tid >> 4, c = (tid & 15) * 4;
      for (int t = 0; t < 4; ++t) As[r][c + t] = ra[t];
    }
    const int r = tid >> 4, c = (tid & 15) * 4;
    for (int t = 0; t < 4; ++t) Bs[r][c + t] = rb[t];
  };
  if (K > 0) load(0);
  for (int k0 = 0; k0 < K; k0 += 16) {
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
}

__device__ inline void store_tile(const v4d (&acc)[2][2], double* __restrict__ C) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int q = 0; q < 4; ++q) {
        const int row = wm + a * 16 + (lane >> 4) + 4 * q;
        const int s = wn + b * 16 + (lane & 15);
        C[(size_t)row * VL + s] = acc[a][b][q];
      }
}

// Plane sums, split over the slots of each plane: workgroup (m tile bx,
// plane L = by, part bz) adds the slots [kb, ke) of its part of plane L:
//   Y[((part nL + L) M2 + m) VL + s] = sum_k Ecat[m][k] P[k][s].
__global__ void __launch_bounds__(256) k_cg_plane_sums(int nslot, int M2, int nlayers, int ksplit,
                                                       const int* __restrict__ plane_off,
                                                       const double* __restrict__ Ecat,
                                                       const double* __restrict__ P,
                                                       double* __restrict__ Y) {
  __shared__ double As[16][68];
  __shared__ double Bs[16][68];
  const int m0 = blockIdx.x * 64, L = blockIdx.y, part = blockIdx.z;
  const int q16 = (plane_off[L + 1] - plane_off[L]) / 16;
  const int kb = plane_off[L] + (q16 * part / ksplit) * 16;
  const int ke = plane_off[L] + (q16 * (part + 1) / ksplit) * 16;
  v4d acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  seg_mfma<false>(acc, Ecat + (size_t)m0 * nslot + kb, nslot, P + (size_t)kb * VL, ke - kb, As, Bs);
  store_tile(acc, Y + (((size_t)part * nlayers + L) * M2 + m0) * VL);
}

// T for every plane: Tcat[(L M2 + 2c) VL + s] = Re, [.. 2c + 1 ..] = Im of
// sum_L' Q_c(L', L) Y(c, L', s) (Y: the sum of its ksplit parts, in order);
// zero rows for padding columns.  Up to MIX_NL planes: one workgroup per
// column with a wave per plane; wave L' sums Y(c, L', .) over its parts into
// LDS, then wave L forms T(c, L, .) in plane order.  More planes: one thread
// per (plane, column, vector).
constexpr int MIX_NL = 16;

__global__ void __launch_bounds__(64 * MIX_NL) k_cg_plane_mix_col(int nlayers, int ncp,
                                                                 int ncolsort, int ksplit,
                                                                 const double2* __restrict__ Q,
                                                                 const double* __restrict__ Y,
                                                                 double* __restrict__ T) {
  __shared__ double2 sy[MIX_NL][VL];
  const int c = blockIdx.x, s = threadIdx.x & 63, L = threadIdx.x >> 6;
  const size_t M2 = 2 * (size_t)ncp;
  double yr = 0.0, yi = 0.0;
  if (c < ncolsort)
    for (int p = 0; p < ksplit; ++p) {
      const double* y = Y + (((size_t)p * nlayers + L) * M2 + 2 * c) * VL + s;
      yr += y[0];
      yi += y[VL];
    }
  sy[L][s] = make_double2(yr, yi);
  __syncthreads();
  double tr = 0.0, ti = 0.0;
  if (c < ncolsort)
    for (int L2 = 0; L2 < nlayers; ++L2) {
      const double2 q = Q[((size_t)c * nlayers + L2) * nlayers + L];
      const double2 y = sy[L2][s];
      tr += q.x * y.x - q.y * y.y;
      ti += q.x * y.y + q.y * y.x;
    }
  T[(L * M2 + 2 * c) * VL + s] = tr;
  T[(L * M2 + 2 * c + 1) * VL + s] = ti;
}

__global__ void k_cg_plane_mix(int nlayers, int ncp, int ncolsort, int ksplit,
                               const double2* __restrict__ Q, const double* __restrict__ Y,
                               double* __restrict__ T) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)nlayers * ncp * VL) return;
  const int s = (int)(e % VL), c = (int)((e / VL) % ncp), L = (int)(e / ((size_t)VL * ncp));
  const size_t M2 = 2 * (size_t)ncp;
  double tr = 0.0, ti = 0.0;
  if (c < ncolsort) {
    for (int L2 = 0; L2 < nlayers; ++L2) {
      double yr = 0.0, yi = 0.0;
      for (int p = 0; p < ksplit; ++p) {
        const double* y = Y + (((size_t)p * nlayers + L2) * M2 + 2 * c) * VL + s;
        yr += y[0];
        yi += y[VL];
      }
      const double2 q = Q[((size_t)c * nlayers + L2) * nlayers + L];
      tr += q.x * yr - q.y * yi;
      ti += q.x * yi + q.y * yr;
    }
  }
  T[(L * M2 + 2 * c) * VL + s] = tr;
  T[(L * M2 + 2 * c + 1) * VL + s] = ti;
}

// Projection and real space per slot tile, one work item per workgroup:
// item = {tile, kind, begin, end, part, plane}.
//   kind 0: k-space projection over columns rows [begin, end) of the phase
//     matrix: Phi_part[tile rows] = Ecat[begin:end, tile]^T T[plane][begin:end];
//   kind 1: real space over the tile's blocks [begin, end) of the 64 x 64
//     block-sparse part R: Phi_part[tile rows] = sum_b R_b P[col tile of b].
// The parts of a tile are added in order by the apply kernel.
__global__ void __launch_bounds__(256) k_cg_tiles(int nslot, int M2,
                                                  const int* __restrict__ items,
                                                  const double* __restrict__ Ecat,
                                                  const double* __restrict__ T,
                                                  const int* __restrict__ bcol,
                                                  const double* __restrict__ bval,
                                                  const double* __restrict__ P,
                                                  double* __restrict__ Phi) {
  __shared__ double As[16][68];
  __shared__ double Bs[16][68];
  const int* it = items + 6 * blockIdx.x;
  const int tile = it[0], kind = it[1], beg = it[2], end = it[3], part = it[4], L = it[5];
  v4d acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  if (kind == 0) {
    seg_mfma<true>(acc, Ecat + (size_t)beg * nslot + (size_t)tile * 64, nslot,
                   T + ((size_t)L * M2 + beg) * VL, end - beg, As, Bs);
  } else {
    for (int b = beg; b < end; ++b)
      seg_mfma<false>(acc, bval + (size_t)b * 64 * 64, 64, P + (size_t)bcol[b] * 64 * VL, 64, As,
                      Bs);
  }
  store_tile(acc, Phi + ((size_t)part * nslot + (size_t)tile * 64) * VL);
}

// The same projection for one right-hand side (lane 0 of T): a matrix-core
// tile would compute 64 lanes to keep one, so the product runs on the vector
// units.  One workgroup per item, as above; its four waves split the item's
// rows into contiguous quarters, lane l takes slot 64 tile + l, and the four
// partial sums are added in wave order.  T's entries are uniform across the
// wave.  Writes lane 0 of the item's Phi rows only.
__global__ void __launch_bounds__(256) k_proj_one(int nslot, int M2, const int* __restrict__ items,
                                                  const double* __restrict__ Ecat,
                                                  const double* __restrict__ T,
                                                  double* __restrict__ Phi) {
  __shared__ double part[4][64];
  const int* it = items + 6 * blockIdx.x;
  const int tile = it[0], beg = it[2], end = it[3], q = it[4], L = it[5];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = beg + (end - beg) * wave / 4, r1 = beg + (end - beg) * (wave + 1) / 4;
  const double* e = Ecat + (size_t)tile * 64 + lane;
  const double* t = T + (size_t)L * M2 * VL;
  double acc = 0.0;
#pragma unroll 8
  for (int r = r0; r < r1; ++r) acc += e[(size_t)r * nslot] * t[(size_t)r * VL];
  part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0)
    Phi[((size_t)q * nslot + (size_t)tile * 64 + lane) * VL] =
        (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// ---- A p and the conjugate-gradient steps ---------------------------------
// Every kernel below runs on the same grid (nblk blocks of CG_WAVES waves),
// so the partials of one are summed by the next over the same block count.

// moments (sum p, sum p x, sum p y, sum p z) of one row into v[0..4)
__device__ inline void add_moments(double* v, double p, int i, const double* __restrict__ ex,
                                   const double* __restrict__ ey, const double* __restrict__ ez) {
  v[0] += p;
  v[1] += p * ex[i];
  v[2] += p * ey[i];
  v[3] += p * ez[i];
}

__device__ inline void store_moments(const double (&m)[4], double* __restrict__ red) {
  const int f[4] = {F_M0, F_M0 + 1, F_M0 + 2, F_M0 + 3};
  store_partials<4>(m, f, red);
}

// Ap = k_e (sum of the Phi parts (k space + real space) + background M0 +
// sum_d c_d r_d M_d) + diag_extra p (operator; DENSE: Ap given), pad slots
// 0; block partials of p.Ap and sum Ap.  M: the moments of p from the kernel
// that wrote p.
template <bool DENSE>
__global__ void __launch_bounds__(CG_BLK) k_cg_apply(
    int nslot, int n, const int* __restrict__ slot_atom, const double* __restrict__ ex,
    const double* __restrict__ ey, const double* __restrict__ ez,
    const double* __restrict__ dextra, int nparts, const double* __restrict__ Phi,
    double background, double cx, double cy, double cz, double ke, const double* __restrict__ P,
    double* __restrict__ AP, double* __restrict__ red) {
  __shared__ double M[4][VL];
  const int s = threadIdx.x & 63;
  if (!DENSE) {
    const int f[4] = {F_M0, F_M0 + 1, F_M0 + 2, F_M0 + 3};
    block_totals<4>(red, gridDim.x, f, M);
  }
  double v[2] = {0.0, 0.0};
  for (Rows w; w.r < nslot; w.r += w.step) {
    const int r = w.r, i = slot_atom[r];
    const double pv = P[(size_t)r * VL + s];
    double ap = 0.0;
    if (i >= 0) {
      if (DENSE) {
        ap = AP[(size_t)r * VL + s];
      } else {
        double phi = 0.0;
        for (int q = 0; q < nparts; ++q) phi += Phi[((size_t)q * nslot + r) * VL + s];
        ap = ke * (phi + (background * M[0][s] +
                          (cx * ex[i] * M[1][s] + cy * ey[i] * M[2][s] + cz * ez[i] * M[3][s]))) +
             dextra[i] * pv;
      }
    }
    if (!DENSE) AP[(size_t)r * VL + s] = ap;
    v[0] += pv * ap;
    v[1] += ap;
  }
  const int f[2] = {F_PAP, F_SAP};
  store_partials<2>(v, f, red);
}

// alpha = r.z / p.Ap (z = M^-1 r, the preconditioned residual, written by
// the preconditioner's npc tile blocks; npc = 0: no preconditioner, z = r)
// for vectors above tolerance (else 0: frozen); x += alpha p,
// r -= alpha (Ap - mean Ap); partials of the new r.r into field
// F_RR + (1 - cur).  Block 0 counts the iteration of each active vector.
__global__ void __launch_bounds__(CG_BLK) k_cg_update(int nslot, int n, int cur, double tol2,
                                                      int npc,
                                                      const int* __restrict__ slot_atom,
                                                      double* __restrict__ X,
                                                      double* __restrict__ R,
                                                      const double* __restrict__ P,
                                                      const double* __restrict__ AP,
                                                      double* __restrict__ red,
                                                      double* __restrict__ scal) {
  __shared__ double t[4][VL];
  __shared__ double z[1][VL];
  const int s = threadIdx.x & 63;
  {
    const int f[4] = {F_PAP, F_SAP, F_RR + cur, F_RRI};
    block_totals<4>(red, gridDim.x, f, t);
  }
  if (npc > 0) {
    const int f[1] = {F_RZ + cur};
    block_totals<1>(red, npc, f, z);
  }
  const double pap = t[0][s], mean = t[1][s] / n, rr = t[2][s], rr0 = t[3][s];
  const double rz = npc > 0 ? z[0][s] : rr;
  const bool active = rr > tol2 * rr0 && pap > 0.0;
  const double a = active ? rz / pap : 0.0;
  if (blockIdx.x == 0 && threadIdx.x < VL && active) scal[S_ITERS * VL + s] += 1.0;
  double v[1] = {0.0};
  for (Rows w; w.r < nslot; w.r += w.step) {
    const int r = w.r;
    if (slot_atom[r] < 0) continue;
    const size_t o = (size_t)r * VL + s;
    X[o] += a * P[o];
    const double rn = R[o] - a * (AP[o] - mean);
    R[o] = rn;
    v[0] += rn * rn;
  }
  const int f[1] = {F_RR + (1 - cur)};
  store_partials<1>(v, f, red);
}

// New direction p = z' - mean(z') + beta p, beta = r'.z' / r.z (npc > 0,
// z' = M^-1 r' in Z from the preconditioner's npc tile blocks) or
// p = r' + beta p, beta = r'.r' / r.r (npc = 0); beta = 0 for frozen vectors
// and on the first call (first = 1, which makes p the first direction);
// moments of the new p.  Block 0 records r'.r' and r0.r0 for the host.
__global__ void __launch_bounds__(CG_BLK) k_cg_dir(int nslot, int n, int cur, double tol2,
                                                   int npc, int first,
                                                   const int* __restrict__ slot_atom,
                                                   const double* __restrict__ ex,
                                                   const double* __restrict__ ey,
                                                   const double* __restrict__ ez,
                                                   const double* __restrict__ R,
                                                   const double* __restrict__ Z,
                                                   double* __restrict__ P, double* __restrict__ red,
                                                   double* __restrict__ scal) {
  __shared__ double t[3][VL];
  __shared__ double u[3][VL];
  const int s = threadIdx.x & 63;
  {
    const int f[3] = {F_RR + cur, F_RR + (1 - cur), F_RRI};
    block_totals<3>(red, gridDim.x, f, t);
  }
  if (npc > 0) {
    const int f[3] = {F_RZ + cur, F_RZ + (1 - cur), F_ZSUM};
    block_totals<3>(red, npc, f, u);
  }
  const double rr = t[0][s], rn = t[1][s], rr0 = t[2][s];
  const bool go = !first && rr > tol2 * rr0;
  const double beta = !go ? 0.0 : npc > 0 ? u[1][s] / u[0][s] : rn / rr;
  const double zmean = npc > 0 ? u[2][s] / n : 0.0;
  if (blockIdx.x == 0 && threadIdx.x < VL) {
    scal[S_RR * VL + s] = rn;
    scal[S_RR0 * VL + s] = rr0;
  }
  const double* src = npc > 0 ? Z : R;
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  for (Rows w; w.r < nslot; w.r += w.step) {
    const int r = w.r, i = slot_atom[r];
    if (i < 0) continue;
    const size_t o = (size_t)r * VL + s;
    const double p = (src[o] - zmean) + beta * P[o];
    P[o] = p;
    add_moments(m, p, i, ex, ey, ez);
  }
  store_moments(m, red);
}

__device__ inline double rhs_value(const void* b, int b_is_f32, int n, int s, int i,
                                   const double* __restrict__ vat) {
  const double bv = b_is_f32 ? (double)reinterpret_cast<const float*>(b)[(size_t)s * n + i]
                             : reinterpret_cast<const double*>(b)[(size_t)s * n + i];
  return bv + vat[i];
}

// partial sums of c = b + v per vector (vectors s < g; b rows n apart, atom order)
__global__ void __launch_bounds__(CG_BLK) k_cg_rhs(int nslot, int n, int g,
                                                   const int* __restrict__ slot_atom,
                                                   const void* b, int b_is_f32,
                                                   const double* __restrict__ vat,
                                                   double* __restrict__ red) {
  const int s = threadIdx.x & 63;
  double v[1] = {0.0};
  for (Rows w; w.r < nslot; w.r += w.step) {
    const int i = slot_atom[w.r];
    if (i >= 0 && s < g) v[0] += rhs_value(b, b_is_f32, n, s, i, vat);
  }
  const int f[1] = {F_SUM};
  store_partials<1>(v, f, red);
}

// x = 0, r = p = c - mean(c) (zero for pads and vectors s >= g); partials of
// r0.r0 (fields F_RR and F_RRI) and of the moments of p; block 0 clears the
// iteration counts and records r0.r0 for the host
__global__ void __launch_bounds__(CG_BLK) k_cg_init(int nslot, int n, int g,
                                                    const int* __restrict__ slot_atom,
                                                    const double* __restrict__ ex,
                                                    const double* __restrict__ ey,
                                                    const double* __restrict__ ez, const void* b,
                                                    int b_is_f32, const double* __restrict__ vat,
                                                    double* __restrict__ X, double* __restrict__ R,
                                                    double* __restrict__ P,
                                                    double* __restrict__ red,
                                                    double* __restrict__ scal) {
  __shared__ double t[1][VL];
  const int s = threadIdx.x & 63;
  {
    const int f[1] = {F_SUM};
    block_totals<1>(red, gridDim.x, f, t);
  }
  const double cm = t[0][s] / n;
  double rr[2] = {0.0, 0.0};
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  for (Rows w; w.r < nslot; w.r += w.step) {
    const int r = w.r, i = slot_atom[r];
    const size_t o = (size_t)r * VL + s;
    double rv = 0.0;
    if (i >= 0 && s < g) rv = rhs_value(b, b_is_f32, n, s, i, vat) - cm;
    X[o] = 0.0;
    R[o] = rv;
    P[o] = rv;
    rr[0] += rv * rv;
    if (i >= 0) add_moments(m, rv, i, ex, ey, ez);
  }
  rr[1] = rr[0];
  const int f[2] = {F_RR, F_RRI};
  store_partials<2>(rr, f, red);
  store_moments(m, red);
  if (blockIdx.x == 0 && threadIdx.x < VL) scal[S_ITERS * VL + s] = 0.0;
}

// P = x (batch x n, atom order) in slot rows, zero elsewhere; moments of it
__global__ void __launch_bounds__(CG_BLK) k_cg_gather(int nslot, int n, int g,
                                                      const int* __restrict__ slot_atom,
                                                      const double* __restrict__ ex,
                                                      const double* __restrict__ ey,
                                                      const double* __restrict__ ez,
                                                      const double* __restrict__ x,
                                                      double* __restrict__ P,
                                                      double* __restrict__ red) {
  const int s = threadIdx.x & 63;
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  for (Rows w; w.r < nslot; w.r += w.step) {
    const int r = w.r, i = slot_atom[r];
    double p = 0.0;
    if (i >= 0 && s < g) p = x[(size_t)s * n + i];
    P[(size_t)r * VL + s] = p;
    if (i >= 0) add_moments(m, p, i, ex, ey, ez);
  }
  store_moments(m, red);
}

// partial sums of x per vector
__global__ void __launch_bounds__(CG_BLK) k_cg_xsum(int nslot, const int* __restrict__ slot_atom,
                                                    const double* __restrict__ X,
                                                    double* __restrict__ red) {
  const int s = threadIdx.x & 63;
  double v[1] = {0.0};
  for (Rows w; w.r < nslot; w.r += w.step)
    if (slot_atom[w.r] >= 0) v[0] += X[(size_t)w.r * VL + s];
  const int f[1] = {F_SUM};
  store_partials<1>(v, f, red);
}

// y (batch x n, atom order) = the slot rows of V, minus the mean of V's
// vectors when `center` (the neutrality projection of the CG iterate)
__global__ void __launch_bounds__(CG_BLK) k_cg_scatter(int nslot, int n, int g, int center,
                                                       const int* __restrict__ slot_atom,
                                                       const double* __restrict__ V,
                                                       const double* __restrict__ red,
                                                       double* __restrict__ y) {
  __shared__ double t[1][VL];
  const int s = threadIdx.x & 63;
  double sh = 0.0;
  if (center) {
    const int f[1] = {F_SUM};
    block_totals<1>(red, gridDim.x, f, t);
    sh = t[0][s] / n;
  }
  for (Rows w; w.r < nslot; w.r += w.step) {
    const int i = slot_atom[w.r];
    if (i >= 0 && s < g) y[(size_t)s * n + i] = V[(size_t)w.r * VL + s] - sh;
  }
}

// electrode totals Qe[s n_e + e] = sum_{i: eid_i = e} q_s[i]; block per vector
__global__ void __launch_bounds__(256) k_cg_totals(int n, const double* __restrict__ q,
                                                   const int* __restrict__ eid, int n_e,
                                                   double* __restrict__ Qe) {
  __shared__ double sh[4];
  const int s = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int e = 0; e < n_e; ++e) {
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256)
      if (eid[i] == e) a += q[(size_t)s * n + i];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (lane == 0) sh[w] = a;
    __syncthreads();
    if (threadIdx.x == 0) Qe[(size_t)s * n_e + e] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
  }
}

// ---- two-level preconditioner ----------------------------------------------
// Additive form: M^-1 r = D_t^-1 r_t on every slot tile t (D_t: A's 64 x 64
// diagonal block of the tile's atoms, identity on pad slots) + Z C^-1 Z^T r,
// Z the coarse basis vectors (the tile constants here) and C = Z^T A Z.
// Both parts are symmetric positive definite, so M^-1 is, and the
// neutral-subspace iteration stays a CG.

// D_t^-1 for every tile (grid: tiles, 256 threads).  D_t from the operator's
// own pieces for atoms i, j of the tile (one plane L):
//   k_e (R_tt(i, j) + sum_c Q_c(L, L) cos(th_i - th_j) + background
//        + sum_d c_d r_id r_jd) + delta_ij diag_extra_i,
// R_tt the tile's real-space + self block (diag_blk[t], -1: none), th the
// in-plane phases of column c; symmetrised, then inverted in LDS by
// Gauss-Jordan elimination (no pivoting: D_t is positive definite).
__global__ void __launch_bounds__(256) k_pc_blocks(
    int nslot, int nlayers, int ncolsort, const int* __restrict__ slot_atom,
    const int* __restrict__ tile_plane, const int* __restrict__ diag_blk,
    const double* __restrict__ bval, const double* __restrict__ Ecat,
    const double2* __restrict__ Q, const double* __restrict__ ex, const double* __restrict__ ey,
    const double* __restrict__ ez, const double* __restrict__ dextra, double background,
    double cx, double cy, double cz, double ke, double* __restrict__ Dinv) {
  __shared__ double D[64][65];
  __shared__ double cs[16][64], sn[16][64], qd[16];
  __shared__ double rk[64], fk[64];
  const int t = blockIdx.x, tid = threadIdx.x, L = tile_plane[t];
  const int i = tid >> 2, j0 = tid & 3;        // entries (i, j0 + 4 u), u = 0..15
  const size_t base = (size_t)t * 64;
  double acc[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) acc[u] = 0.0;
  for (int c0 = 0; c0 < ncolsort; c0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int cc = e >> 6, sl = e & 63, c = c0 + cc;
      const bool in = c < ncolsort;
      cs[cc][sl] = in ? Ecat[(size_t)(2 * c) * nslot + base + sl] : 0.0;
      sn[cc][sl] = in ? Ecat[(size_t)(2 * c + 1) * nslot + base + sl] : 0.0;
    }
    if (tid < 16) {
      const int c = c0 + tid;
      qd[tid] = c < ncolsort ? Q[((size_t)c * nlayers + L) * nlayers + L].x : 0.0;
    }
    __syncthreads();
    for (int cc = 0; cc < 16; ++cc) {
      const double ci = qd[cc] * cs[cc][i], si = qd[cc] * sn[cc][i];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] += ci * cs[cc][j0 + 4 * u] + si * sn[cc][j0 + 4 * u];
    }
    __syncthreads();
  }
  const int ai = slot_atom[base + i], bd = diag_blk[t];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int j = j0 + 4 * u, aj = slot_atom[base + j];
    double d = i == j ? 1.0 : 0.0;
    if (ai >= 0 && aj >= 0) {
      const double rs = bd >= 0 ? bval[(size_t)bd * 4096 + i * 64 + j] : 0.0;
      d = ke * ((acc[u] + rs) +
                (background + (cx * ex[ai] * ex[aj] + cy * ey[ai] * ey[aj] + cz * ez[ai] * ez[aj])));
      if (i == j) d += dextra[ai];
    }
    D[i][j] = d;
  }
  __syncthreads();
  double sym[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) sym[u] = 0.5 * (D[i][j0 + 4 * u] + D[j0 + 4 * u][i]);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 16; ++u) D[i][j0 + 4 * u] = sym[u];
  __syncthreads();
  for (int k = 0; k < 64; ++k) {
    if (tid < 64) {
      const double piv = D[k][k];
      rk[tid] = (tid == k ? 1.0 : D[k][tid]) / piv;
      fk[tid] = tid == k ? 0.0 : D[tid][k];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int j = j0 + 4 * u;
      D[i][j] = i == k ? rk[j] : (j == k ? 0.0 : D[i][j]) - fk[i] * rk[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int j = j0 + 4 * u;
    Dinv[(size_t)t * 4096 + i * 64 + j] = 0.5 * (D[i][j] + D[j][i]);
  }
}

// Coarse space: K basis functions per tile, phi[slot * 3 + c] (c < K; 0 on
// pads): the tile's constant and, for K = 3, the in-plane offsets from the
// tile's centre (scaled; 0 where a tile is too small or too thin for them).
// Coarse column j = tile * K + c.

// P = coarse columns j0 .. j0 + g - 1 (vector s: column j0 + s) on the CG
// grid, with the moments of P for the operator
__global__ void __launch_bounds__(CG_BLK) k_pc_basis(int nslot, int K, int j0, int g,
                                                     const int* __restrict__ slot_atom,
                                                     const double* __restrict__ phi,
                                                     const double* __restrict__ ex,
                                                     const double* __restrict__ ey,
                                                     const double* __restrict__ ez,
                                                     double* __restrict__ P,
                                                     double* __restrict__ red) {
  const int s = threadIdx.x & 63;
  const int j = j0 + s, jt = j / K, jc = j % K;
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  for (Rows w; w.r < nslot; w.r += w.step) {
    const int r = w.r, i = slot_atom[r];
    const double p = (i >= 0 && s < g && (r >> 6) == jt) ? phi[(size_t)r * 3 + jc] : 0.0;
    P[(size_t)r * VL + s] = p;
    if (i >= 0) add_moments(m, p, i, ex, ey, ez);
  }
  store_moments(m, red);
}

// sums over the 64 rows of tile blockIdx.x of V (256 threads; fixed order:
// wave w adds rows w, w + 4, ..., then the 4 waves in order), weighted by
// the basis function c (phi = nullptr: weight 1); thread s < 64 gets the sum
// of vector s
__device__ inline double tile_sum(const double* __restrict__ V, double (*sh)[VL],
                                  const double* __restrict__ phi = nullptr, int c = 0,
                                  int tile = -1) {
  const int s = threadIdx.x & 63, w = threadIdx.x >> 6;
  const size_t base = (size_t)(tile >= 0 ? tile : blockIdx.x) * 64;
  double a = 0.0;
  for (int r = w; r < 64; r += 4)
    a += (phi ? phi[(base + r) * 3 + c] : 1.0) * V[(base + r) * VL + s];
  __syncthreads();
  sh[w][s] = a;
  __syncthreads();
  return (sh[0][s] + sh[1][s]) + (sh[2][s] + sh[3][s]);
}

// C[(t K + c) ld + j0 + s] = sum over tile t of phi_c V's vector s (s < g):
// rows of Z^T A Z from V = A (coarse columns j0 ..)
__global__ void __launch_bounds__(256) k_pc_coarse_cols(int ld, int K, int j0, int g,
                                                        const double* __restrict__ phi,
                                                        const double* __restrict__ V,
                                                        double* __restrict__ C) {
  __shared__ double sh[4][VL];
  const int s = threadIdx.x;
  for (int c = 0; c < K; ++c) {
    const double a = tile_sum(V, sh, phi, c);
    if (s < g) C[((size_t)blockIdx.x * K + c) * ld + j0 + s] = a;
  }
}

// B = (C + C^T) / 2 on the leading T x T block (row stride ld)
__global__ void k_pc_sym(int T, int ld, const double* __restrict__ C, double* __restrict__ B) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)T * T) return;
  const int i = (int)(e / T), j = (int)(e % T);
  const double v = 0.5 * (C[(size_t)i * ld + j] + C[(size_t)j * ld + i]);
  // a basis function that is zero on its tile leaves a zero row and column:
  // a unit diagonal there keeps C invertible and that coarse entry inert
  B[(size_t)i * ld + j] = (i == j && v == 0.0) ? 1.0 : v;
}

// one Gauss-Jordan step (pivot k, no pivoting: C is positive definite) from
// A into B on the leading T x T block; T steps turn C into C^-1
__global__ void k_pc_gj_step(int T, int ld, int k, const double* __restrict__ A,
                             double* __restrict__ B) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)T * T) return;
  const int i = (int)(e / T), j = (int)(e % T);
  const size_t o = (size_t)i * ld + j;
  const double rkj = (j == k ? 1.0 : A[(size_t)k * ld + j]) / A[(size_t)k * ld + k];
  B[o] = i == k ? rkj : (j == k ? 0.0 : A[o]) - A[(size_t)i * ld + k] * rkj;
}

// Local part, per tile (grid: tiles, 256 threads): Z_t = D_t^-1 R_t on the
// matrix cores, and the tile sums Z^T R
__global__ void __launch_bounds__(256) k_pc_local(const double* __restrict__ Dinv,
                                                  const double* __restrict__ R,
                                                  double* __restrict__ Z,
                                                  double* __restrict__ ZtR) {
  __shared__ double As[16][68];
  __shared__ double Bs[16][68];
  __shared__ double sh[4][VL];
  const size_t t = blockIdx.x;
  v4d acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  seg_mfma<false>(acc, Dinv + t * 4096, 64, R + t * 64 * VL, 64, As, Bs);
  store_tile(acc, Z + t * 64 * VL);
  const double a = tile_sum(R, sh);
  if (threadIdx.x < VL) ZtR[t * VL + threadIdx.x] = a;
}

// Coarse part and the sums the direction needs, per tile (grid: tiles,
// CG_WAVES waves): Z_t += (C^-1 Z^T R)_t on real slots (pads 0); block
// partials of r.z into field fnew and of sum z into F_ZSUM.
__global__ void __launch_bounds__(CG_BLK) k_pc_coarse(int T, int ld, int fnew,
                                                      const int* __restrict__ slot_atom,
                                                      const double* __restrict__ Cinv,
                                                      const double* __restrict__ ZtR,
                                                      const double* __restrict__ R,
                                                      double* __restrict__ Z,
                                                      double* __restrict__ red) {
  __shared__ double sh[CG_WAVES][VL];
  __shared__ double cc[VL];
  const int t = blockIdx.x, s = threadIdx.x & 63, w = threadIdx.x >> 6;
  double a = 0.0;
  for (int u = w; u < T; u += CG_WAVES) a += Cinv[(size_t)t * ld + u] * ZtR[(size_t)u * VL + s];
  sh[w][s] = a;
  __syncthreads();
  if (threadIdx.x < VL) cc[s] = sum16(sh, s);
  __syncthreads();
  double v[2] = {0.0, 0.0};
  for (int r = t * 64 + w; r < t * 64 + 64; r += CG_WAVES) {
    const size_t o = (size_t)r * VL + s;
    const double z = slot_atom[r] >= 0 ? Z[o] + cc[s] : 0.0;
    Z[o] = z;
    v[0] += R[o] * z;
    v[1] += z;
  }
  const int f[2] = {fnew, F_ZSUM};
  store_partials<2>(v, f, red);
}

// Balancing form of the two-level preconditioner (the coarse correction on
// both sides of the tile-block smoother B = blockdiag(D_t^-1)):
//   M^-1 r = Q r + (I - Q A) B (I - A Q) r,   Q = Z C^-1 Z^T,
// symmetric positive definite like the additive form.  With the set-up
// products DAZ = B A Z (slots x ld) and H = C^-1 + C^-1 (A Z)^T DAZ C^-1 it is
//   t = Z^T r,  y = DAZ^T r,  w = C^-1 t,  g = H t - C^-1 y,
//   z = B r - DAZ w + Z g,
// two products with DAZ per iteration (the coarse arrays are ld x 64, ld
// the coarse-space dimension rounded up to 64, zero beyond it).

// y parts (KA): Ypart[(part ld + m) VL + s] = sum over the slots of part of
// DAZ[slot][m] R[slot][s]; grid (ld / 64, parts), tile-aligned slot ranges
__global__ void __launch_bounds__(256) k_bnn_y(int ntile, int ld, const double* __restrict__ DAZ,
                                               const double* __restrict__ R,
                                               double* __restrict__ Ypart) {
  __shared__ double As[16][68];
  __shared__ double Bs[16][68];
  const int m0 = blockIdx.x * 64, part = blockIdx.y, np = gridDim.y;
  const int kb = ntile * part / np * 64, ke = ntile * (part + 1) / np * 64;
  v4d acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  seg_mfma<true>(acc, DAZ + (size_t)kb * ld + m0, ld, R + (size_t)kb * VL, ke - kb, As, Bs);
  store_tile(acc, Ypart + ((size_t)part * ld + m0) * VL);
}

// -y = minus the sum of the parts, t = Z^T r (the basis-weighted tile sums of
// R; 0 beyond the ntile * K coarse columns); grid ld, 256 threads
__global__ void __launch_bounds__(256) k_bnn_sum(int ntile, int K, int ld, int nparts,
                                                 const double* __restrict__ phi,
                                                 const double* __restrict__ Ypart,
                                                 const double* __restrict__ R,
                                                 double* __restrict__ Yn, double* __restrict__ Tt) {
  __shared__ double sh[4][VL];
  __shared__ double sy[4][VL];
  const int u = blockIdx.x, s = threadIdx.x & 63, w = threadIdx.x >> 6;
  double a = 0.0;
  for (int p = w; p < nparts; p += 4) a += Ypart[((size_t)p * ld + u) * VL + s];
  sy[w][s] = a;
  // uniform branch: tile_sum synchronises inside
  const double tt = u < ntile * K ? tile_sum(R, sh, K > 1 ? phi : nullptr, u % K, u / K) : 0.0;
  __syncthreads();
  if (threadIdx.x < VL) {
    Yn[(size_t)u * VL + s] = -((sy[0][s] + sy[1][s]) + (sy[2][s] + sy[3][s]));
    Tt[(size_t)u * VL + s] = tt;
  }
}

// coarse vectors (KB) on the matrix cores, 64 coarse rows per workgroup:
// blockIdx.y = 0: Wn = -C^-1 t; 1: G = H t + C^-1 (-y); grid (ld / 64, 2,
// parts): part p adds the coarse columns [p ld / parts, (p + 1) ld / parts)
// (multiples of 16) into its own slice of Out (parts > 1), or writes Wn and G
// directly (parts = 1)
__global__ void __launch_bounds__(256) k_bnn_coarse(int ld, const double* __restrict__ Cinv,
                                                    const double* __restrict__ H,
                                                    const double* __restrict__ Tt,
                                                    const double* __restrict__ Yn,
                                                    double* __restrict__ Wn,
                                                    double* __restrict__ G,
                                                    double* __restrict__ Out) {
  __shared__ double As[16][68];
  __shared__ double Bs[16][68];
  const size_t u0 = (size_t)blockIdx.x * 64;
  const int np = gridDim.z, p = blockIdx.z;
  const int q16 = ld / 16, kb = q16 * p / np * 16, kl = q16 * (p + 1) / np * 16 - kb;
  v4d acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  if (blockIdx.y == 0) {
    seg_mfma<false>(acc, Cinv + u0 * ld + kb, ld, Tt + (size_t)kb * VL, kl, As, Bs);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) acc[a][b] = -acc[a][b];
  } else {
    seg_mfma<false>(acc, H + u0 * ld + kb, ld, Tt + (size_t)kb * VL, kl, As, Bs);
    seg_mfma<false>(acc, Cinv + u0 * ld + kb, ld, Yn + (size_t)kb * VL, kl, As, Bs);
  }
  if (np == 1)
    store_tile(acc, (blockIdx.y == 0 ? Wn : G) + u0 * VL);
  else
    store_tile(acc, Out + (((size_t)p * 2 + blockIdx.y) * ld + u0) * VL);
}

// The same for short coarse spaces (ld <= 128), on the vector units with a
// workgroup per coarse row (more workgroups than the matrix-core form has):
// grid ld, CG_WAVES waves
__global__ void __launch_bounds__(CG_BLK) k_bnn_coarse_rows(int ld, const double* __restrict__ Cinv,
                                                            const double* __restrict__ H,
                                                            const double* __restrict__ Tt,
                                                            const double* __restrict__ Yn,
                                                            double* __restrict__ Wn,
                                                            double* __restrict__ G) {
  __shared__ double s1[CG_WAVES][VL];
  __shared__ double s2[CG_WAVES][VL];
  const int u = blockIdx.x, s = threadIdx.x & 63, w = threadIdx.x >> 6;
  double a = 0.0, b = 0.0;
  for (int v = w; v < ld; v += CG_WAVES) {
    const double c = Cinv[(size_t)u * ld + v], h = H[(size_t)u * ld + v];
    const double tv = Tt[(size_t)v * VL + s];
    a += c * tv;
    b += h * tv + c * Yn[(size_t)v * VL + s];
  }
  s1[w][s] = a;
  s2[w][s] = b;
  __syncthreads();
  if (threadIdx.x < VL) {
    Wn[(size_t)u * VL + s] = -sum16(s1, s);
    G[(size_t)u * VL + s] = sum16(s2, s);
  }
}

// Wn and G from the parts of k_bnn_coarse (added in part order)
__global__ void k_bnn_coarse_sum(int ld, int np, const double* __restrict__ Out,
                                 double* __restrict__ Wn, double* __restrict__ G) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x, m = (size_t)ld * VL;
  if (e >= 2 * m) return;
  const int y = (int)(e / m);
  const size_t o = e % m;
  double a = 0.0;
  for (int p = 0; p < np; ++p) a += Out[((size_t)p * 2 + y) * m + o];
  (y == 0 ? Wn : G)[o] = a;
}

// z per tile (KC): Z_t = D_t^-1 R_t + DAZ_t Wn + sum_c phi_c g_(t K + c) on
// real slots (pads 0),
// on the matrix cores; block partials of r.z into field fnew and of sum z
// into F_ZSUM (grid: tiles, 256 threads)
__global__ void __launch_bounds__(256) k_bnn_z(int ld, int K, int fnew,
                                               const int* __restrict__ slot_atom,
                                               const double* __restrict__ phi,
                                               const double* __restrict__ Dinv,
                                               const double* __restrict__ DAZ,
                                               const double* __restrict__ Wn,
                                               const double* __restrict__ G,
                                               const double* __restrict__ R,
                                               double* __restrict__ Z, double* __restrict__ red) {
  __shared__ double As[16][68];
  __shared__ double Bs[16][68];
  __shared__ double zs[64][65];
  __shared__ double sh[2][4][VL];
  const size_t t = blockIdx.x;
  v4d acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  seg_mfma<false>(acc, Dinv + t * 4096, 64, R + t * 64 * VL, 64, As, Bs);
  seg_mfma<false>(acc, DAZ + t * 64 * ld, ld, Wn, ld, As, Bs);
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int q = 0; q < 4; ++q)
          zs[wm + a * 16 + (lane >> 4) + 4 * q][wn + b * 16 + (lane & 15)] = acc[a][b][q];
  }
  __syncthreads();
  const int s = threadIdx.x & 63, w = threadIdx.x >> 6;
  double gt[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < K; ++c) gt[c] = G[(t * K + c) * VL + s];
  double rz = 0.0, zsum = 0.0;
  for (int r = w; r < 64; r += 4) {
    const size_t o = (t * 64 + r) * VL + s;
    double cg = gt[0];
    if (K > 1) {
      const double* ph = phi + (t * 64 + r) * 3;
      cg = gt[0] * ph[0];
      for (int c = 1; c < K; ++c) cg += gt[c] * ph[c];
    }
    const double z = slot_atom[t * 64 + r] >= 0 ? zs[r][s] + cg : 0.0;
    Z[o] = z;
    rz += R[o] * z;
    zsum += z;
  }
  sh[0][w][s] = rz;
  sh[1][w][s] = zsum;
  __syncthreads();
  if (threadIdx.x < VL) {
    red[(t * CG_RED + fnew) * VL + s] = (sh[0][0][s] + sh[0][1][s]) + (sh[0][2][s] + sh[0][3][s]);
    red[(t * CG_RED + F_ZSUM) * VL + s] =
        (sh[1][0][s] + sh[1][1][s]) + (sh[1][2][s] + sh[1][3][s]);
  }
}

}  // namespace

int cg_blocks(int nslot, int cap) { return std::max(1, std::min(cap, nslot / CG_WAVES)); }

int cg_scalar_row(int which) { return which == 0 ? S_RR : which == 1 ? S_RR0 : S_ITERS; }

void launch_ell_count(hipStream_t st, int nslot, int jchunks, const int* slot_atom,
                      const Buffers& b, double Lx, double Ly, double Lz, double rc, int* cnt) {
  const int chunk = (nslot + jchunks - 1) / jchunks;
  // alpha, eta_ee and the self term do not enter the count
  hipLaunchKernelGGL(k_ell_pass<false>, dim3((nslot + 255) / 256, jchunks), dim3(256), 0, st,
                     nslot, chunk, 0, slot_atom, b.ex, b.ey, b.ez, Lx, Ly, Lz, rc, 1.0, 1.0, 0.0,
                     cnt, nullptr, nullptr);
}

void launch_ell_fill(hipStream_t st, int nslot, int jchunks, int width, const int* slot_atom,
                     const int* off, const Buffers& b, double Lx, double Ly, double Lz, double rc,
                     double alpha, double eta_ee, double diag_self, int* col, double* val) {
  const size_t total = (size_t)width * nslot;
  hipLaunchKernelGGL(k_ell_init, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, width,
                     total, col, val);
  const int chunk = (nslot + jchunks - 1) / jchunks;
  hipLaunchKernelGGL(k_ell_pass<true>, dim3((nslot + 255) / 256, jchunks), dim3(256), 0, st, nslot,
                     chunk, width, slot_atom, b.ex, b.ey, b.ez, Lx, Ly, Lz, rc, alpha, eta_ee,
                     diag_self, const_cast<int*>(off), col, val);
}

void launch_cg_ephase(hipStream_t st, int nslot, int ncp, int ncolsort, const int* slot_atom,
                      const Buffers& b, double* Ecat) {
  hipLaunchKernelGGL(k_cg_ephase, dim3((nslot + 255) / 256, ncp), dim3(256), 0, st, nslot,
                     ncolsort, slot_atom, b.sc_nx, b.sc_ny, b.efx, b.efy, Ecat);
}

void launch_cg_plane_sums(hipStream_t st, int nslot, int ncp, int nlayers, int ksplit,
                          const int* plane_off, const double* Ecat, const double* P, double* Y) {
  hipLaunchKernelGGL(k_cg_plane_sums, dim3(2 * ncp / 64, nlayers, ksplit), dim3(256), 0, st, nslot,
                     2 * ncp, nlayers, ksplit, plane_off, Ecat, P, Y);
}

void launch_cg_plane_mix(hipStream_t st, int ncp, int ncolsort, int nlayers, int ksplit,
                         const double2* Q, const double* Y, double* T) {
  if (nlayers <= MIX_NL) {
    hipLaunchKernelGGL(k_cg_plane_mix_col, dim3(ncp), dim3(64 * nlayers), 0, st, nlayers, ncp,
                       ncolsort, ksplit, Q, Y, T);
    return;
  }
  const size_t tot = (size_t)nlayers * ncp * VL;
  hipLaunchKernelGGL(k_cg_plane_mix, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     nlayers, ncp, ncolsort, ksplit, Q, Y, T);
}

void launch_cg_tiles(hipStream_t st, int nitems, int nslot, int ncp, const int* items,
                     const double* Ecat, const double* T, const int* bcol, const double* bval,
                     const double* P, double* Phi) {
  hipLaunchKernelGGL(k_cg_tiles, dim3(nitems), dim3(256), 0, st, nslot, 2 * ncp, items, Ecat, T,
                     bcol, bval, P, Phi);
}

void launch_proj_one(hipStream_t st, int nitems, int nslot, int ncp, const int* items,
                     const double* Ecat, const double* T, double* Phi) {
  hipLaunchKernelGGL(k_proj_one, dim3(nitems), dim3(256), 0, st, nslot, 2 * ncp, items, Ecat, T,
                     Phi);
}

void launch_cg_apply(hipStream_t st, bool dense, int nblk, int nslot, int n, const int* slot_atom,
                     const Buffers& b, int nparts, const double* Phi, double background,
                     const double* cdip, double ke, const double* P, double* AP, double* red) {
  if (dense)
    hipLaunchKernelGGL(k_cg_apply<true>, dim3(nblk), dim3(CG_BLK), 0, st, nslot, n, slot_atom,
                       b.ex, b.ey, b.ez, b.dextra, nparts, Phi, background, cdip[0], cdip[1],
                       cdip[2], ke, P, AP, red);
  else
    hipLaunchKernelGGL(k_cg_apply<false>, dim3(nblk), dim3(CG_BLK), 0, st, nslot, n, slot_atom,
                       b.ex, b.ey, b.ez, b.dextra, nparts, Phi, background, cdip[0], cdip[1],
                       cdip[2], ke, P, AP, red);
}

void launch_cg_update(hipStream_t st, int nblk, int nslot, int n, int cur, double tol2, int npc,
                      const int* slot_atom, double* X, double* R, const double* P,
                      const double* AP, double* red, double* scal) {
  hipLaunchKernelGGL(k_cg_update, dim3(nblk), dim3(CG_BLK), 0, st, nslot, n, cur, tol2, npc,
                     slot_atom, X, R, P, AP, red, scal);
}

void launch_cg_dir(hipStream_t st, int nblk, int nslot, int n, int cur, double tol2, int npc,
                   int first, const int* slot_atom, const Buffers& b, const double* R,
                   const double* Z, double* P, double* red, double* scal) {
  hipLaunchKernelGGL(k_cg_dir, dim3(nblk), dim3(CG_BLK), 0, st, nslot, n, cur, tol2, npc, first,
                     slot_atom, b.ex, b.ey, b.ez, R, Z, P, red, scal);
}

void launch_cg_init(hipStream_t st, int nblk, int nslot, int n, int g, const int* slot_atom,
                    const Buffers& b, const void* bsrc, int b_is_f32, double* X, double* R,
                    double* P, double* red, double* scal) {
  hipLaunchKernelGGL(k_cg_rhs, dim3(nblk), dim3(CG_BLK), 0, st, nslot, n, g, slot_atom, bsrc,
                     b_is_f32, b.vat, red);
  hipLaunchKernelGGL(k_cg_init, dim3(nblk), dim3(CG_BLK), 0, st, nslot, n, g, slot_atom, b.ex,
                     b.ey, b.ez, bsrc, b_is_f32, b.vat, X, R, P, red, scal);
}

void launch_cg_gather(hipStream_t st, int nblk, int nslot, int n, int g, const int* slot_atom,
                      const Buffers& b, const double* x, double* P, double* red) {
  hipLaunchKernelGGL(k_cg_gather, dim3(nblk), dim3(CG_BLK), 0, st, nslot, n, g, slot_atom, b.ex,
                     b.ey, b.ez, x, P, red);
}

void launch_cg_scatter(hipStream_t st, int nblk, int nslot, int n, int g, const int* slot_atom,
                       const double* V, double* y) {
  hipLaunchKernelGGL(k_cg_scatter, dim3(nblk), dim3(CG_BLK), 0, st, nslot, n, g, 0, slot_atom, V,
                     nullptr, y);
}

void launch_cg_finish(hipStream_t st, int nblk, int nslot, int n, int g, const int* slot_atom,
                      const double* X, double* red, const int* eid, int n_e, double* q,
                      double* Qe) {
  hipLaunchKernelGGL(k_cg_xsum, dim3(nblk), dim3(CG_BLK), 0, st, nslot, slot_atom, X, red);
  hipLaunchKernelGGL(k_cg_scatter, dim3(nblk), dim3(CG_BLK), 0, st, nslot, n, g, 1, slot_atom, X,
                     red, q);
  if (Qe) hipLaunchKernelGGL(k_cg_totals, dim3(g), dim3(256), 0, st, n, q, eid, n_e, Qe);
}

void launch_pc_blocks(hipStream_t st, int ntile, int nslot, int nlayers, int ncolsort,
                      const int* slot_atom, const int* tile_plane, const int* diag_blk,
                      const double* bval, const double* Ecat, const double2* Q, const Buffers& b,
                      double background, const double* cdip, double ke, double* Dinv) {
  hipLaunchKernelGGL(k_pc_blocks, dim3(ntile), dim3(256), 0, st, nslot, nlayers, ncolsort,
                     slot_atom, tile_plane, diag_blk, bval, Ecat, Q, b.ex, b.ey, b.ez, b.dextra,
                     background, cdip[0], cdip[1], cdip[2], ke, Dinv);
}

void launch_pc_basis(hipStream_t st, int nblk, int nslot, int K, int j0, int g,
                     const int* slot_atom, const double* phi, const Buffers& b, double* P,
                     double* red) {
  hipLaunchKernelGGL(k_pc_basis, dim3(nblk), dim3(CG_BLK), 0, st, nslot, K, j0, g, slot_atom, phi,
                     b.ex, b.ey, b.ez, P, red);
}

void launch_pc_coarse_cols(hipStream_t st, int ntile, int ld, int K, int j0, int g,
                           const double* phi, const double* V, double* C) {
  hipLaunchKernelGGL(k_pc_coarse_cols, dim3(ntile), dim3(256), 0, st, ld, K, j0, g, phi, V, C);
}

double* launch_pc_invert(hipStream_t st, int ntile, int ld, double* C, double* W) {
  const size_t tot = (size_t)ntile * ntile;
  const dim3 grid((unsigned)((tot + 255) / 256));
  hipLaunchKernelGGL(k_pc_sym, grid, dim3(256), 0, st, ntile, ld, C, W);
  double* a = W;
  double* o = C;
  for (int k = 0; k < ntile; ++k) {
    hipLaunchKernelGGL(k_pc_gj_step, grid, dim3(256), 0, st, ntile, ld, k, a, o);
    std::swap(a, o);
  }
  return a;
}

void launch_pc_apply(hipStream_t st, int ntile, int ld, int parity, const int* slot_atom,
                     const double* Dinv, const double* Cinv, const double* R, double* Z,
                     double* ZtR, double* red) {
  hipLaunchKernelGGL(k_pc_local, dim3(ntile), dim3(256), 0, st, Dinv, R, Z, ZtR);
  hipLaunchKernelGGL(k_pc_coarse, dim3(ntile), dim3(CG_BLK), 0, st, ntile, ld, F_RZ + parity,
                     slot_atom, Cinv, ZtR, R, Z, red);
}

void launch_bnn_apply(hipStream_t st, int ntile, int K, int ld, int nparts, int cparts,
                      int parity, const int* slot_atom, const double* phi, const double* Dinv,
                      const double* DAZ, const double* Cinv, const double* H, const double* R,
                      double* Z, double* Ypart, double* Yn, double* Tt, double* Wn, double* G,
                      double* Cpart, double* red) {
  hipLaunchKernelGGL(k_bnn_y, dim3(ld / 64, nparts), dim3(256), 0, st, ntile, ld, DAZ, R, Ypart);
  hipLaunchKernelGGL(k_bnn_sum, dim3(ld), dim3(256), 0, st, ntile, K, ld, nparts, phi, Ypart, R,
                     Yn, Tt);
  if (ld <= 128)
    hipLaunchKernelGGL(k_bnn_coarse_rows, dim3(ld), dim3(CG_BLK), 0, st, ld, Cinv, H, Tt, Yn, Wn, G);
  else
    hipLaunchKernelGGL(k_bnn_coarse, dim3(ld / 64, 2, cparts), dim3(256), 0, st, ld, Cinv, H, Tt,
                       Yn, Wn, G, Cpart);
  if (ld > 128 && cparts > 1) {
    const size_t tot = (size_t)2 * ld * VL;
    hipLaunchKernelGGL(k_bnn_coarse_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, ld,
                       cparts, Cpart, Wn, G);
  }
  hipLaunchKernelGGL(k_bnn_z, dim3(ntile), dim3(256), 0, st, ld, K, F_RZ + parity, slot_atom, phi,
                     Dinv, DAZ, Wn, G, R, Z, red);
}

}  // namespace cpm
