// Matrix-free elastance operator and the projected conjugate-gradient solve.
//
// The charges minimise the electrostatic energy under charge neutrality
// (Sec. II.A; the conjugate-gradient route it names as the alternative to
// inverting A): q solves A q = b + v + mu e with e^T q = 0.  Conjugate
// gradients on the neutral subspace (projector P = I - e e^T / n) need only
// products A p, never A^-1 or S, so the memory stays O(n) per vector plus the
// fixed electrode tables:
//   * real space + Gaussian self term: a fixed sparse matrix (every pair with
//     some periodic image within r_c), kept in ELL form and evaluated with the
//     same expression as the dense assembly;
//   * k space for electrodes on z planes: with E_j(c) = e^{i (kx x_j + ky y_j)}
//     and Q_c(L, L') = sum_n 2W(c, n) e^{i n kz1 (z_L - z_L')},
//       (A_k p)_i = k_e sum_c Re[conj(E_i(c)) T(c, L_i)],
//       T(c, L) = sum_L' Q_c(L', L) Y(c, L'),  Y(c, L') = sum_{j in L'} E_j(c) p_j,
//     (the planar regrouping of A's k-space term, applied to a vector);
//   * background -pi/(V alpha^2) (sum p) and the geometry's dipole term
//     sum_d c_d r_id (sum_j r_jd p_j) from four moments of p;
//   * the optional per-atom diagonal.
// Every reduction runs in a fixed order (block partials summed in block
// order), so results do not depend on scheduling.
#include "cpm_internal.h"

namespace cpm {

namespace {

constexpr int CG_BLK = 256;
// block partial fields: p.Ap, sum Ap, r.r (two slots, alternating), r0.r0, sum
constexpr int F_PAP = 0, F_SAP = 1, F_RR = 2, F_RRI = 4, F_SUM = 5;
static_assert(F_SUM < CG_RED, "partial fields");

inline int cg_blocks(int n) { return (n + CG_BLK - 1) / CG_BLK; }

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sums over 256 threads: park() leaves each wave's sum of v in
// sh[slot][wave]; after a barrier, parked(slot) = (w0 + w1) + (w2 + w3).
// Deterministic (lane 0's butterfly order, fixed wave order).
__device__ inline void park(double v, int slot, double (*sh)[4]) {
  const double t = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[slot][threadIdx.x >> 6] = t;
}

__device__ inline double parked(int slot, const double (*sh)[4]) {
  return (sh[slot][0] + sh[slot][1]) + (sh[slot][2] + sh[slot][3]);
}

// sum over the blocks of vector s of partial field f (block order)
__device__ inline double sum_partials(const double* __restrict__ red, int nblk, int s, int f) {
  double a = 0.0;
  for (int k = 0; k < nblk; ++k) a += red[((size_t)s * nblk + k) * CG_RED + f];
  return a;
}

// ---- real-space + self part of A in ELL form ----------------------------------
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

// One pass over the j chunk of row i.  FILL = false counts the entries
// (cnt[chunk n + i]); FILL = true writes them from off[chunk n + i] on, never
// past kend (the next chunk's offset, or the width for the last chunk).  Both
// passes run this same code, so they take the same in-range decisions.
template <bool FILL>
__global__ void __launch_bounds__(256) k_ell_pass(int n, int chunk, int width,
                                                  const double* __restrict__ ex,
                                                  const double* __restrict__ ey,
                                                  const double* __restrict__ ez, double Lx,
                                                  double Ly, double Lz, double rc, double alpha,
                                                  double eta_ee, double diag_self,
                                                  int* __restrict__ cnt, int* __restrict__ col,
                                                  double* __restrict__ val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, ch = blockIdx.y;
  if (i >= n) return;
  const int j0 = ch * chunk, j1 = min(n, j0 + chunk);
  const double xi = ex[i], yi = ey[i], zi = ez[i];
  size_t k = FILL ? (size_t)cnt[(size_t)ch * n + i] : 0;
  const size_t kend = FILL ? (ch + 1 < (int)gridDim.y ? (size_t)cnt[(size_t)(ch + 1) * n + i]
                                                      : (size_t)width)
                           : 0;
  for (int j = j0; j < j1; ++j) {
    double s;
    const int c = pair_images(xi - ex[j], yi - ey[j], zi - ez[j], Lx, Ly, Lz, rc, alpha, eta_ee, &s);
    if (j == i || c > 0) {
      if (FILL && k < kend) {
        col[k * n + i] = j;
        val[k * n + i] = (j == i) ? s + diag_self : s;
      }
      ++k;
    }
  }
  if (!FILL) cnt[(size_t)ch * n + i] = (int)k;
}

__global__ void k_ell_init(int n, size_t total, int* __restrict__ col, double* __restrict__ val) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  col[e] = (int)(e % n);
  val[e] = 0.0;
}

// ---- k-space part: plane sums, plane mixing -----------------------------------
// Y[(c nL + L) g + s] = sum over the atoms j of plane L of E_j(c) p_s[j].  One
// wave per (column, plane); the plane's atoms are the slots
// [plane_off[L], plane_off[L + 1]) of the atom map (-1 pads).
__global__ void __launch_bounds__(64) k_op_plane_sums(int g, int n, int nlayers,
                                                      const int* __restrict__ plane_off,
                                                      const int* __restrict__ amap,
                                                      const double2* __restrict__ E,
                                                      const double* __restrict__ P, int ldp,
                                                      double2* __restrict__ Y) {
  const int c = blockIdx.x, L = blockIdx.y, lane = threadIdx.x;
  double ar[CG_MAXG], ai[CG_MAXG];
#pragma unroll
  for (int s = 0; s < CG_MAXG; ++s) { ar[s] = 0.0; ai[s] = 0.0; }
  const double2* Ec = E + (size_t)c * n;
  for (int t = plane_off[L] + lane; t < plane_off[L + 1]; t += 64) {
    const int j = amap[t];
    if (j < 0) continue;
    const double2 e = Ec[j];
#pragma unroll
    for (int s = 0; s < CG_MAXG; ++s)
      if (s < g) {
        const double pv = P[(size_t)s * ldp + j];
        ar[s] += e.x * pv;
        ai[s] += e.y * pv;
      }
  }
  double2* y = Y + ((size_t)c * nlayers + L) * g;
#pragma unroll
  for (int s = 0; s < CG_MAXG; ++s)
    if (s < g) {
      const double r = wave_sum(ar[s]), im = wave_sum(ai[s]);
      if (lane == 0) y[s] = make_double2(r, im);
    }
}

// T[(c nL + L) g + s] = sum_L' Q_c(L', L) Y[(c nL + L') g + s]
__global__ void k_op_plane_mix(int g, int nlayers, int ncolsort, const double2* __restrict__ Q,
                               const double2* __restrict__ Y, double2* __restrict__ T) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncolsort * nlayers * g) return;
  const int s = e % g, L = (e / g) % nlayers, c = e / (g * nlayers);
  double tr = 0.0, ti = 0.0;
  for (int L2 = 0; L2 < nlayers; ++L2) {
    const double2 q = Q[((size_t)c * nlayers + L2) * nlayers + L];
    const double2 y = Y[((size_t)c * nlayers + L2) * g + s];
    tr += q.x * y.x - q.y * y.y;
    ti += q.x * y.y + q.y * y.x;
  }
  T[e] = make_double2(tr, ti);
}

// moments of each vector per block: mom[((s nblk + blk) 4 + d)] for
// d = 0: sum p, 1..3: sum p r_d (raw coordinates)
__global__ void __launch_bounds__(256) k_op_moments(int g, int n, const double* __restrict__ ex,
                                                    const double* __restrict__ ey,
                                                    const double* __restrict__ ez,
                                                    const double* __restrict__ P, int ldp,
                                                    double* __restrict__ mom) {
  __shared__ double sh[4 * CG_MAXG][4];
  const int i = blockIdx.x * CG_BLK + threadIdx.x, nblk = gridDim.x;
  double x = 0, y = 0, z = 0;
  if (i < n) { x = ex[i]; y = ey[i]; z = ez[i]; }
  for (int s = 0; s < g; ++s) {
    const double pv = i < n ? P[(size_t)s * ldp + i] : 0.0;
    park(pv, 4 * s, sh);
    park(pv * x, 4 * s + 1, sh);
    park(pv * y, 4 * s + 2, sh);
    park(pv * z, 4 * s + 3, sh);
  }
  __syncthreads();
  if ((int)threadIdx.x < 4 * g) {
    const int s = threadIdx.x / 4, d = threadIdx.x % 4;
    mom[((size_t)s * nblk + blockIdx.x) * 4 + d] = parked(threadIdx.x, sh);
  }
}

// Ap = k_e (k-space + ELL real space + background sum p + sum_d c_d r_d M_d)
// + diag_extra p, and the block partials of p.Ap and sum Ap.
__global__ void __launch_bounds__(256) k_op_final(
    int g, int n, int ldp, int cgroups, const double* __restrict__ phik, int width,
    const int* __restrict__ ecol, const double* __restrict__ evals,
    const double* __restrict__ mom, const double* __restrict__ ex, const double* __restrict__ ey,
    const double* __restrict__ ez, double background, double cx, double cy, double cz, double ke,
    const double* __restrict__ dextra, const double* __restrict__ P, double* __restrict__ AP,
    double* __restrict__ red) {
  __shared__ double sM[4 * CG_MAXG];
  __shared__ double sh[2 * CG_MAXG][4];
  const int i = blockIdx.x * CG_BLK + threadIdx.x, nblk = gridDim.x;
  if ((int)threadIdx.x < 4 * g) {
    const int s = threadIdx.x / 4, d = threadIdx.x % 4;
    double a = 0.0;
    for (int k = 0; k < nblk; ++k) a += mom[((size_t)s * nblk + k) * 4 + d];
    sM[threadIdx.x] = a;
  }
  __syncthreads();
  double acc[CG_MAXG];
#pragma unroll
  for (int s = 0; s < CG_MAXG; ++s) acc[s] = 0.0;
  if (i < n) {
    for (int k = 0; k < width; ++k) {
      const int j = ecol[(size_t)k * n + i];
      const double a = evals[(size_t)k * n + i];
#pragma unroll
      for (int s = 0; s < CG_MAXG; ++s)
        if (s < g) acc[s] += a * P[(size_t)s * ldp + j];
    }
  }
  double x = 0, y = 0, z = 0, de = 0;
  if (i < n) { x = ex[i]; y = ey[i]; z = ez[i]; de = dextra[i]; }
#pragma unroll
  for (int s = 0; s < CG_MAXG; ++s) {
    if (s < g) {
      double pv = 0.0, ap = 0.0;
      if (i < n) {
        double pk = 0.0;
        for (int r = 0; r < cgroups; ++r) pk += phik[((size_t)r * g + s) * n + i];
        const double* M = sM + 4 * s;
        pv = P[(size_t)s * ldp + i];
        ap = ke * ((pk + acc[s]) + (background * M[0] + (cx * x * M[1] + cy * y * M[2] +
                                                         cz * z * M[3]))) + de * pv;
        AP[(size_t)s * ldp + i] = ap;
      }
      park(pv * ap, 2 * s, sh);
      park(ap, 2 * s + 1, sh);
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < 2 * g) {
    const int s = threadIdx.x / 2, f = threadIdx.x % 2 ? F_SAP : F_PAP;
    red[((size_t)s * nblk + blockIdx.x) * CG_RED + f] = parked(threadIdx.x, sh);
  }
}

// ---- conjugate-gradient steps (grid: blocks of 256 atoms, all vectors) -------
// partials of p.Ap and sum Ap for an Ap computed elsewhere (dense A)
__global__ void __launch_bounds__(256) k_cg_dots(int g, int n, int ldp, const double* __restrict__ P,
                                                 const double* __restrict__ AP,
                                                 double* __restrict__ red) {
  __shared__ double sh[2 * CG_MAXG][4];
  const int i = blockIdx.x * CG_BLK + threadIdx.x, nblk = gridDim.x;
  for (int s = 0; s < g; ++s) {
    const double ap = i < n ? AP[(size_t)s * ldp + i] : 0.0;
    const double pv = i < n ? P[(size_t)s * ldp + i] : 0.0;
    park(pv * ap, 2 * s, sh);
    park(ap, 2 * s + 1, sh);
  }
  __syncthreads();
  if ((int)threadIdx.x < 2 * g) {
    const int s = threadIdx.x / 2, f = threadIdx.x % 2 ? F_SAP : F_PAP;
    red[((size_t)s * nblk + blockIdx.x) * CG_RED + f] = parked(threadIdx.x, sh);
  }
}

__device__ inline double rhs_value(const void* b, int b_is_f32, int n, int s, int i,
                                   const double* __restrict__ vat) {
  const double bv = b_is_f32 ? (double)reinterpret_cast<const float*>(b)[(size_t)s * n + i]
                             : reinterpret_cast<const double*>(b)[(size_t)s * n + i];
  return bv + vat[i];
}

// partial sums of c = b + v
__global__ void __launch_bounds__(256) k_cg_rhs_sum(int g, int n, const void* b, int b_is_f32,
                                                    const double* __restrict__ vat,
                                                    double* __restrict__ red) {
  __shared__ double sh[CG_MAXG][4];
  const int i = blockIdx.x * CG_BLK + threadIdx.x, nblk = gridDim.x;
  for (int s = 0; s < g; ++s) park(i < n ? rhs_value(b, b_is_f32, n, s, i, vat) : 0.0, s, sh);
  __syncthreads();
  if ((int)threadIdx.x < g)
    red[((size_t)threadIdx.x * nblk + blockIdx.x) * CG_RED + F_SUM] = parked(threadIdx.x, sh);
}

// x = 0, r = p = P c; partials of r.r into slot 0 and the initial field;
// iteration counters cleared
__global__ void __launch_bounds__(256) k_cg_init(int g, int n, int ldp, const void* b, int b_is_f32,
                                                 const double* __restrict__ vat,
                                                 double* __restrict__ red, double* __restrict__ X,
                                                 double* __restrict__ R, double* __restrict__ P,
                                                 double* __restrict__ stat) {
  __shared__ double smean[CG_MAXG];
  __shared__ double sh[CG_MAXG][4];
  const int i = blockIdx.x * CG_BLK + threadIdx.x, nblk = gridDim.x;
  if ((int)threadIdx.x < g) {
    smean[threadIdx.x] = sum_partials(red, nblk, threadIdx.x, F_SUM) / n;
    if (blockIdx.x == 0) stat[3 * threadIdx.x + 2] = 0.0;
  }
  __syncthreads();
  for (int s = 0; s < g; ++s) {
    double r = 0.0;
    if (i < n) {
      r = rhs_value(b, b_is_f32, n, s, i, vat) - smean[s];
      X[(size_t)s * ldp + i] = 0.0;
      R[(size_t)s * ldp + i] = r;
      P[(size_t)s * ldp + i] = r;
    }
    park(r * r, s, sh);
  }
  __syncthreads();
  if ((int)threadIdx.x < g) {
    double* o = red + ((size_t)threadIdx.x * nblk + blockIdx.x) * CG_RED;
    o[F_RR] = parked(threadIdx.x, sh);
    o[F_RRI] = parked(threadIdx.x, sh);
  }
}

// alpha = r.r / p.Ap for vectors still above tolerance (else 0: frozen);
// x += alpha p, r -= alpha P Ap; partials of the new r.r into the other slot
__global__ void __launch_bounds__(256) k_cg_update(int g, int n, int ldp, int cur, double tol2,
                                                   double* __restrict__ red,
                                                   double* __restrict__ X, double* __restrict__ R,
                                                   const double* __restrict__ P,
                                                   const double* __restrict__ AP,
                                                   double* __restrict__ stat) {
  __shared__ double salpha[CG_MAXG], smean[CG_MAXG];
  __shared__ double sh[CG_MAXG][4];
  const int i = blockIdx.x * CG_BLK + threadIdx.x, nblk = gridDim.x;
  if ((int)threadIdx.x < g) {
    const int s = threadIdx.x;
    const double pap = sum_partials(red, nblk, s, F_PAP), sap = sum_partials(red, nblk, s, F_SAP);
    const double rr = sum_partials(red, nblk, s, F_RR + cur);
    const double rr0 = sum_partials(red, nblk, s, F_RRI);
    const bool active = rr > tol2 * rr0 && pap > 0.0;
    salpha[s] = active ? rr / pap : 0.0;
    smean[s] = sap / n;
    if (blockIdx.x == 0 && active) stat[3 * s + 2] += 1.0;
  }
  __syncthreads();
  for (int s = 0; s < g; ++s) {
    double r = 0.0;
    if (i < n) {
      const size_t o = (size_t)s * ldp + i;
      const double a = salpha[s];
      X[o] += a * P[o];
      r = R[o] - a * (AP[o] - smean[s]);
      R[o] = r;
    }
    park(r * r, s, sh);
  }
  __syncthreads();
  if ((int)threadIdx.x < g)
    red[((size_t)threadIdx.x * nblk + blockIdx.x) * CG_RED + F_RR + (1 - cur)] = parked(threadIdx.x, sh);
}

// beta = r'.r' / r.r (0 for frozen vectors); p = r' + beta p
__global__ void __launch_bounds__(256) k_cg_dir(int g, int n, int ldp, int cur, double tol2,
                                                const double* __restrict__ red,
                                                const double* __restrict__ R,
                                                double* __restrict__ P) {
  __shared__ double sbeta[CG_MAXG];
  const int i = blockIdx.x * CG_BLK + threadIdx.x, nblk = gridDim.x;
  if ((int)threadIdx.x < g) {
    const int s = threadIdx.x;
    const double rr = sum_partials(red, nblk, s, F_RR + cur);
    const double rn = sum_partials(red, nblk, s, F_RR + (1 - cur));
    const double rr0 = sum_partials(red, nblk, s, F_RRI);
    sbeta[s] = rr > tol2 * rr0 ? rn / rr : 0.0;
  }
  __syncthreads();
  if (i >= n) return;
  for (int s = 0; s < g; ++s) {
    const size_t o = (size_t)s * ldp + i;
    P[o] = R[o] + sbeta[s] * P[o];
  }
}

// stat[3 s] = r.r (slot cur), stat[3 s + 1] = r0.r0
__global__ void k_cg_status(int g, int nblk, int cur, const double* __restrict__ red,
                            double* __restrict__ stat) {
  const int s = threadIdx.x;
  if (s >= g) return;
  stat[3 * s] = sum_partials(red, nblk, s, F_RR + cur);
  stat[3 * s + 1] = sum_partials(red, nblk, s, F_RRI);
}

__global__ void __launch_bounds__(256) k_cg_xsum(int g, int n, int ldp, const double* __restrict__ X,
                                                 double* __restrict__ red) {
  __shared__ double sh[CG_MAXG][4];
  const int i = blockIdx.x * CG_BLK + threadIdx.x, nblk = gridDim.x;
  for (int s = 0; s < g; ++s) park(i < n ? X[(size_t)s * ldp + i] : 0.0, s, sh);
  __syncthreads();
  if ((int)threadIdx.x < g)
    red[((size_t)threadIdx.x * nblk + blockIdx.x) * CG_RED + F_SUM] = parked(threadIdx.x, sh);
}

// q = x - mean(x) (the neutrality projection, exact up to rounding)
__global__ void __launch_bounds__(256) k_cg_finish(int g, int n, int ldp,
                                                   const double* __restrict__ X,
                                                   const double* __restrict__ red,
                                                   double* __restrict__ q) {
  __shared__ double smean[CG_MAXG];
  const int i = blockIdx.x * CG_BLK + threadIdx.x, nblk = gridDim.x;
  if ((int)threadIdx.x < g) smean[threadIdx.x] = sum_partials(red, nblk, threadIdx.x, F_SUM) / n;
  __syncthreads();
  if (i >= n) return;
  for (int s = 0; s < g; ++s) q[(size_t)s * n + i] = X[(size_t)s * ldp + i] - smean[s];
}

// electrode totals Qe[s n_e + e] = sum_{i: eid_i = e} q_s[i]; block per vector
__global__ void __launch_bounds__(256) k_cg_totals(int n, const double* __restrict__ q,
                                                   const int* __restrict__ eid, int n_e,
                                                   double* __restrict__ Qe) {
  __shared__ double sh[1][4];
  const int s = blockIdx.x;
  for (int e = 0; e < n_e; ++e) {
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += CG_BLK)
      if (eid[i] == e) a += q[(size_t)s * n + i];
    park(a, 0, sh);
    __syncthreads();
    if (threadIdx.x == 0) Qe[(size_t)s * n_e + e] = parked(0, sh);
    __syncthreads();
  }
}

}  // namespace

void launch_ell_count(hipStream_t st, int n, int jchunks, const Buffers& b, double Lx, double Ly,
                      double Lz, double rc, int* cnt) {
  const int chunk = (n + jchunks - 1) / jchunks;
  // alpha, eta_ee and the self term do not enter the count
  hipLaunchKernelGGL(k_ell_pass<false>, dim3((n + 255) / 256, jchunks), dim3(256), 0, st, n, chunk,
                     0, b.ex, b.ey, b.ez, Lx, Ly, Lz, rc, 1.0, 1.0, 0.0, cnt, nullptr, nullptr);
}

// off: per-chunk starting offsets (the exclusive prefix of the counts along
// each row, chunk-major like the counts)
void launch_ell_fill(hipStream_t st, int n, int jchunks, int width, const int* off,
                     const Buffers& b, double Lx, double Ly, double Lz, double rc, double alpha,
                     double eta_ee, double diag_self, int* col, double* val) {
  const size_t total = (size_t)width * n;
  hipLaunchKernelGGL(k_ell_init, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, total,
                     col, val);
  const int chunk = (n + jchunks - 1) / jchunks;
  hipLaunchKernelGGL(k_ell_pass<true>, dim3((n + 255) / 256, jchunks), dim3(256), 0, st, n, chunk,
                     width, b.ex, b.ey, b.ez, Lx, Ly, Lz, rc, alpha, eta_ee, diag_self,
                     const_cast<int*>(off), col, val);
}

void launch_op_apply(cpm_ctx* c, int g, const double* P, double* AP) {
  const Buffers& b = c->b;
  hipStream_t st = c->stream;
  const int n = c->n, ldp = c->npad, nL = c->nlayers, nc = c->ncolsort, nblk = cg_blocks(n);
  hipLaunchKernelGGL(k_op_plane_sums, dim3(nc, nL), dim3(64), 0, st, g, n, nL, b.plane_off, b.amap,
                     b.ephase, P, ldp, b.cgY);
  const int tot = nc * nL * g;
  hipLaunchKernelGGL(k_op_plane_mix, dim3((tot + 255) / 256), dim3(256), 0, st, g, nL, nc, b.Qpair,
                     b.cgY, b.cgT);
  launch_layer_project_groups(st, g, n, nc, nL, c->op_cgroups, b.ephase, b.layer_of, b.cgT,
                              b.cgphi);
  hipLaunchKernelGGL(k_op_moments, dim3(nblk), dim3(CG_BLK), 0, st, g, n, b.ex, b.ey, b.ez, P, ldp,
                     b.cgmom);
  hipLaunchKernelGGL(k_op_final, dim3(nblk), dim3(CG_BLK), 0, st, g, n, ldp, c->op_cgroups,
                     b.cgphi, c->ell_width, b.ell_col, b.ell_val, b.cgmom, b.ex, b.ey, b.ez,
                     c->op_background, c->cdip[0], c->cdip[1], c->cdip[2], c->ke, b.dextra, P, AP,
                     b.cgred);
}

void launch_cg_dots(hipStream_t st, int g, int n, int ldp, const double* P, const double* AP,
                    double* red) {
  hipLaunchKernelGGL(k_cg_dots, dim3(cg_blocks(n)), dim3(CG_BLK), 0, st, g, n, ldp, P, AP, red);
}

void launch_cg_init(hipStream_t st, int g, int n, int ldp, const void* b, int b_is_f32,
                    const double* vat, double* red, double* X, double* R, double* P, double* stat) {
  hipLaunchKernelGGL(k_cg_rhs_sum, dim3(cg_blocks(n)), dim3(CG_BLK), 0, st, g, n, b, b_is_f32, vat,
                     red);
  hipLaunchKernelGGL(k_cg_init, dim3(cg_blocks(n)), dim3(CG_BLK), 0, st, g, n, ldp, b, b_is_f32, vat,
                     red, X, R, P, stat);
}

void launch_cg_update(hipStream_t st, int g, int n, int ldp, int cur, double tol2,
                      double* red, double* X, double* R, const double* P, const double* AP,
                      double* stat) {
  hipLaunchKernelGGL(k_cg_update, dim3(cg_blocks(n)), dim3(CG_BLK), 0, st, g, n, ldp, cur, tol2,
                     red, X, R, P, AP, stat);
}

void launch_cg_dir(hipStream_t st, int g, int n, int ldp, int cur, double tol2, const double* red,
                   const double* R, double* P) {
  hipLaunchKernelGGL(k_cg_dir, dim3(cg_blocks(n)), dim3(CG_BLK), 0, st, g, n, ldp, cur, tol2, red,
                     R, P);
}

void launch_cg_status(hipStream_t st, int g, int n, int cur, const double* red, double* stat) {
  hipLaunchKernelGGL(k_cg_status, dim3(1), dim3(64), 0, st, g, cg_blocks(n), cur, red, stat);
}

void launch_cg_finish(hipStream_t st, int g, int n, int ldp, const double* X, double* red,
                      const int* eid, int n_e, double* q, double* Qe) {
  hipLaunchKernelGGL(k_cg_xsum, dim3(cg_blocks(n)), dim3(CG_BLK), 0, st, g, n, ldp, X, red);
  hipLaunchKernelGGL(k_cg_finish, dim3(cg_blocks(n)), dim3(CG_BLK), 0, st, g, n, ldp, X, red, q);
  if (Qe) hipLaunchKernelGGL(k_cg_totals, dim3(g), dim3(CG_BLK), 0, st, n, q, eid, n_e, Qe);
}

}  // namespace cpm
