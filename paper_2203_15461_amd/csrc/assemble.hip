// Assembly of the elastance matrix A in FP64 (ELECTRODE paper, Eq. 2: A is
// fixed while the electrodes do not move, so it is built once).
//
//   A_ij = k_e { sum_t [erfc(alpha r) - erfc(eta_ee r)] / r      (real space)
//              + sum_{k in K+} 2 W(k) cos(k.(R_i - R_j))          (k space)
//              - pi / (V alpha^2)                                  (background)
//              + delta_ij (sqrt(2) eta - 2 alpha) / sqrt(pi)       (Gaussian self)
//              + (4 pi / V) z_i z_j }                              (slab, Eq. 12)
//          + delta_ij x_i                                          (optional diagonal)
//
// eta_ee = eta / sqrt(2) is the Gaussian-Gaussian width.  The real-space sum
// runs over all in-plane images t with 0 < r < r_c; the slab clearance
// (slab_factor - 1) h > r_c means no z image is ever inside r_c.  The
// k-space sum is a rank-2|K+| symmetric product T T^T with
// T_i = sqrt(2 k_e W(k)) [cos(k.R_i), sin(k.R_i)], done on FP64 MFMA by the
// dense kernels; this file builds T chunk by chunk.
#include "cpm_internal.h"

namespace cpm {

__global__ void k_prep_electrodes(int n, const double* __restrict__ xyz, double Lx, double Ly,
                                  double Lz, double* ex, double* ey, double* ez, double* fx,
                                  double* fy, double* fz) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // raw coordinates (the dipole terms need them; pair distances use the
  // nearest image), fractional x and y wrapped into [0, 1)
  const double x = xyz[3 * i + 0], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
  ex[i] = x; ey[i] = y; ez[i] = z;
  fx[i] = x / Lx - floor(x / Lx); fy[i] = y / Ly - floor(y / Ly); fz[i] = z / Lz;
}

void launch_prep_electrodes(hipStream_t st, int n, const double* xyz, double Lx, double Ly,
                            double Lz, Buffers& b) {
  hipLaunchKernelGGL(k_prep_electrodes, dim3((n + 255) / 256), dim3(256), 0, st, n, xyz, Lx, Ly,
                     Lz, b.ex, b.ey, b.ez, b.efx, b.efy, b.efz);
}

// Real-space, self, background and dipole parts of A, lower triangle only
// (the upper triangle is mirrored after the k-space product).  Padding rows
// and columns (index >= n) get the identity.
__global__ void __launch_bounds__(256) k_real_space_A(
    int n, int npad, const double* __restrict__ ex, const double* __restrict__ ey,
    const double* __restrict__ ez, double Lx, double Ly, double Lz, double rc, double alpha,
    double eta_ee, double diag_self, double background, double cx, double cy, double cz,
    double ke, const double* __restrict__ diag_extra, double* __restrict__ A) {
  if (blockIdx.x > blockIdx.y) return;               // strictly upper tile
  const int j = blockIdx.x * 16 + threadIdx.x;
  const int i = blockIdx.y * 16 + threadIdx.y;
  if (i >= npad || j >= npad || j > i) return;
  double val;
  if (i >= n || j >= n) {
    val = (i == j) ? 1.0 : 0.0;
  } else {
    const double invLx = 1.0 / Lx, invLy = 1.0 / Ly, invLz = 1.0 / Lz, rc2 = rc * rc;
    const double r2_gauss = eta_ee > alpha ? 45.0 / (eta_ee * eta_ee - alpha * alpha) : 1e300;
    double dx = ex[i] - ex[j], dy = ey[i] - ey[j], dz = ez[i] - ez[j];
    dx -= Lx * rint(dx * invLx);
    dy -= Ly * rint(dy * invLy);
    dz -= Lz * rint(dz * invLz);
    double sum = 0.0;
    if (fabs(dz) < rc) {               // dz is the nearest image: no image is closer
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
              // erfc(eta_ee r) is below FP64 rounding of the difference once
              // (eta_ee^2 - alpha^2) r^2 > 45 (erfc(x) <= e^{-x^2})
              if (r < rc) sum += (r2 > r2_gauss ? erfc(alpha * r) : erfc(alpha * r) - erfc(eta_ee * r)) / r;
            }
          }
        }
      }
    }
    val = sum + background + cx * ex[i] * ex[j] + cy * ey[i] * ey[j] + cz * ez[i] * ez[j];
    if (i == j) val += diag_self;
    val *= ke;
    if (i == j && diag_extra) val += diag_extra[i];
  }
  A[(size_t)i * npad + j] = val;
}

void launch_real_space_A(hipStream_t st, int n, int npad, const Buffers& b, double Lx, double Ly,
                         double Lz, double rc, double alpha, double eta_ee, double diag_self,
                         double background, const double* cdip, double ke,
                         const double* diag_extra, double* A) {
  const int nt = (npad + 15) / 16;
  dim3 grid(nt, nt), block(16, 16);
  hipLaunchKernelGGL(k_real_space_A, grid, block, 0, st, n, npad, b.ex, b.ey, b.ez, Lx, Ly, Lz, rc,
                     alpha, eta_ee, diag_self, background, cdip[0], cdip[1], cdip[2], ke,
                     diag_extra, A);
}

// Phase table for k indices [k0, k0 + kc) of the flat k list:
//   T[i][2c] = sqrt(k_e 2W) cos(k.R_i),  T[i][2c+1] = sqrt(k_e 2W) sin(k.R_i).
// Phases come from fractional coordinates: k.R = 2 pi (nx fx + ny fy + nz fz),
// reduced to [-1/2, 1/2] turns in FP64 before the sincospi.
__global__ void k_phase_table(int n, int npad, int k0, int kc, int nk, const int* __restrict__ knx,
                              const int* __restrict__ kny, const int* __restrict__ knz,
                              const double* __restrict__ w2, const double* __restrict__ fx,
                              const double* __restrict__ fy, const double* __restrict__ fz,
                              double ke, double* __restrict__ T) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (c >= kc) return;
  const int t = k0 + c;
  double cv = 0.0, sv = 0.0;
  if (i < n && t < nk) {
    double th = knx[t] * fx[i] + kny[t] * fy[i] + knz[t] * fz[i];
    th -= rint(th);
    double s, co;
    sincospi(2.0 * th, &s, &co);
    const double amp = sqrt(ke * w2[t]);
    cv = amp * co;
    sv = amp * s;
  }
  double2* row = reinterpret_cast<double2*>(T + (size_t)i * (2 * kc));
  row[c] = make_double2(cv, sv);
}

void launch_phase_table(hipStream_t st, int n, int npad, int k0, int kc, int nk, const Buffers& b,
                        double ke, double* table) {
  dim3 grid((kc + 127) / 128, npad), block(128);
  hipLaunchKernelGGL(k_phase_table, grid, block, 0, st, n, npad, k0, kc, nk, b.knx,
                     b.kny, b.knz, b.w2, b.efx, b.efy, b.efz, ke, table);
}

// ---------------------------------------------------------------------------
// k-space part of A for electrodes on z planes.  For a (k_x, k_y) column c
// and atoms i, j on planes L_i, L_j the column's terms regroup exactly as
//   sum_n 2W(c, n) cos(k . (R_i - R_j)) = Re[E_i(c) conj(E_j(c)) Q_c(L_i, L_j)],
//   E_i(c) = e^{i (kx x_i + ky y_i)},  Q_c(L, L') = sum_n 2W(c, n) e^{i n kz1 (z_L - z_L')},
// so for the atoms of plane L the rows of A gain G_L F^L with
//   G_L[i][2c] = cos th_c(i), G_L[i][2c+1] = -sin th_c(i)   (rows in plane order),
//   F^L[2c][j] = Re, F^L[2c+1][j] = Im of conj(E_j(c)) Q_c(L, L_j):
// one MFMA GEMM with K = 2 x (number of columns) per plane instead of the
// rank-2|K+| product.
// ---------------------------------------------------------------------------

// Q[(c * nlayers + L) * nlayers + L'] = Q_c(L, L'), thread per (c, L, L')
__global__ void k_plane_pair_weights(int ncolsort, int nlayers, const int* __restrict__ sc_lo,
                                     const int* __restrict__ sc_len,
                                     const int* __restrict__ sc_koff,
                                     const double* __restrict__ w2,
                                     const double* __restrict__ layer_fz,
                                     double2* __restrict__ Q) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncolsort * nlayers * nlayers) return;
  const int c = e / (nlayers * nlayers), L = (e / nlayers) % nlayers, L2 = e % nlayers;
  const double dfz = layer_fz[L] - layer_fz[L2];
  double qr = 0.0, qi = 0.0;
  for (int t = 0; t < sc_len[c]; ++t) {
    double th = (sc_lo[c] + t) * dfz;
    th -= rint(th);
    double sn, cs;
    sincospi(2.0 * th, &sn, &cs);
    const double w = w2[sc_koff[c] + t];
    qr += w * cs;
    qi += w * sn;
  }
  Q[e] = make_double2(qr, qi);
}

void launch_plane_pair_weights(hipStream_t st, int ncolsort, int nlayers, const int* sc_lo,
                                const int* sc_len, const int* sc_koff, const double* w2,
                                const double* layer_fz, double2* Q) {
  const int tot = ncolsort * nlayers * nlayers;
  hipLaunchKernelGGL(k_plane_pair_weights, dim3((tot + 255) / 256), dim3(256), 0, st, ncolsort,
                     nlayers, sc_lo, sc_len, sc_koff, w2, layer_fz, Q);
}

// G (nmap x ldG, rows in atom-map order, -1 rows and columns >= 2 ncolsort zero)
__global__ void k_build_G(int nmap, int ncolsort, int ldG, const int* __restrict__ amap,
                          const int* __restrict__ sc_nx, const int* __restrict__ sc_ny,
                          const double* __restrict__ fx, const double* __restrict__ fy,
                          double* __restrict__ G) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (2 * c >= ldG) return;
  const int a = amap[r];
  double cs = 0.0, sn = 0.0;
  if (a >= 0 && c < ncolsort) {
    double th = sc_nx[c] * fx[a] + sc_ny[c] * fy[a];
    th -= rint(th);
    sincospi(2.0 * th, &sn, &cs);
  }
  reinterpret_cast<double2*>(G + (size_t)r * ldG)[c] = make_double2(cs, -sn);
}

void launch_build_G(hipStream_t st, int nmap, int ncolsort, int ldG, const int* amap,
                    const int* sc_nx, const int* sc_ny, const Buffers& b, double* G) {
  dim3 grid((ldG / 2 + 127) / 128, nmap), block(128);
  hipLaunchKernelGGL(k_build_G, grid, block, 0, st, nmap, ncolsort, ldG, amap, sc_nx, sc_ny, b.efx,
                     b.efy, G);
}

// F^L (ldG x npad): column j < n holds conj(E_j(c)) Q_c(L, L_j) as (Re, Im)
// in rows (2c, 2c + 1); padding zero
__global__ void k_build_F(int L, int n, int npad, int nlayers, int ncolsort, int ldG,
                          const int* __restrict__ sc_nx, const int* __restrict__ sc_ny,
                          const double* __restrict__ fx, const double* __restrict__ fy,
                          const int* __restrict__ layer_of, const double2* __restrict__ Q,
                          double* __restrict__ F) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (j >= npad) return;
  double fr = 0.0, fi = 0.0;
  if (j < n && c < ncolsort) {
    double th = sc_nx[c] * fx[j] + sc_ny[c] * fy[j];
    th -= rint(th);
    double sn, cs;
    sincospi(2.0 * th, &sn, &cs);
    const double2 q = Q[((size_t)c * nlayers + L) * nlayers + layer_of[j]];
    // (cs - i sn) (q.x + i q.y)
    fr = cs * q.x + sn * q.y;
    fi = cs * q.y - sn * q.x;
  }
  F[(size_t)(2 * c) * npad + j] = fr;
  F[(size_t)(2 * c + 1) * npad + j] = fi;
}

void launch_build_F(hipStream_t st, int L, int n, int npad, int nlayers, int ncolsort, int ldG,
                    const int* sc_nx, const int* sc_ny, const Buffers& b, const double2* Q,
                    double* F) {
  dim3 grid((npad + 255) / 256, ldG / 2), block(256);
  hipLaunchKernelGGL(k_build_F, grid, block, 0, st, L, n, npad, nlayers, ncolsort, ldG, sc_nx,
                     sc_ny, b.efx, b.efy, b.layer_of, Q, F);
}

// Copy the lower triangle onto the upper one (tiled transpose through LDS).
__global__ void k_mirror_lower(int npad, double* A) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x, by = blockIdx.y;         // source tile (row by, col bx), by > bx
  if (by <= bx) {
    if (by == bx) {                                    // diagonal tile: in place
      const int r = by * 32 + threadIdx.y, c = bx * 32 + threadIdx.x;
      for (int yy = 0; yy < 32; yy += 8) {
        const int rr = r + yy;
        if (c > rr) A[(size_t)rr * npad + c] = A[(size_t)c * npad + rr];
      }
    }
    return;
  }
  for (int yy = 0; yy < 32; yy += 8)
    tile[threadIdx.y + yy][threadIdx.x] =
        A[(size_t)(by * 32 + threadIdx.y + yy) * npad + bx * 32 + threadIdx.x];
  __syncthreads();
  for (int yy = 0; yy < 32; yy += 8)
    A[(size_t)(bx * 32 + threadIdx.y + yy) * npad + by * 32 + threadIdx.x] =
        tile[threadIdx.x][threadIdx.y + yy];
}

void launch_mirror_lower(hipStream_t st, int npad, double* A) {
  dim3 grid(npad / 32, npad / 32), block(32, 8);
  hipLaunchKernelGGL(k_mirror_lower, grid, block, 0, st, npad, A);
}

}  // namespace cpm
