// Host side of libcpm: argument validation, the k-space set, device buffers
// and the launch sequences behind each C-ABI entry point (include/cpm.h).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include <string>
#include "cpm_internal.h"

using namespace cpm;

namespace {

cpm_status fail(cpm_ctx* c, cpm_status st, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return st;
}

#define HIP_TRY(ctx, expr)                                                               \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail((ctx), CPM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Device allocations of a context are recorded with their sizes, so that
// CPM_INFO_WORKSPACE stays exact across frees and reallocations.
template <typename T>
cpm_status dalloc(cpm_ctx* c, T** p, size_t count) {
  if (*p) return CPM_OK;
  void* q = nullptr;
  const size_t bytes = count * sizeof(T) > 0 ? count * sizeof(T) : 16;
  if (hipMalloc(&q, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, CPM_ENOMEM, "device allocation of %zu bytes failed", count * sizeof(T));
  }
  c->bytes += bytes;
  c->alloc_sizes[q] = bytes;
  ++c->alloc_gen;
  *p = static_cast<T*>(q);
  return CPM_OK;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

template <typename T>
void dfree(cpm_ctx* c, T*& p) {
  if (p) {
    ++c->alloc_gen;
    auto it = c->alloc_sizes.find((const void*)p);
    if (it != c->alloc_sizes.end()) {
      c->bytes -= it->second;
      c->alloc_sizes.erase(it);
    }
  }
  dfree(p);
}

// Work arrays whose sizes follow the geometry: an allocation that is large
// enough is kept (no hipFree / hipMalloc, which would wait for the device,
// when a rebuild keeps the sizes), a smaller one is replaced.
template <typename T>
cpm_status dalloc_cap(cpm_ctx* c, T** p, size_t count) {
  if (*p) {
    const auto it = c->alloc_sizes.find((const void*)*p);
    const size_t need = count * sizeof(T) > 0 ? count * sizeof(T) : 16;
    if (it != c->alloc_sizes.end() && it->second >= need) return CPM_OK;
    dfree(c, *p);
  }
  return dalloc(c, p, count);
}

#define TRY(expr)                  \
  do {                             \
    cpm_status s_ = (expr);        \
    if (s_ != CPM_OK) return s_;   \
  } while (0)

// check for launch errors without synchronising
cpm_status launched(cpm_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, CPM_EHIP, "%s: %s", what, hipGetErrorString(e));
  return CPM_OK;
}

// ---- asynchronous inversion ------------------------------------------------
// cpm_invert with CPM_INVERT_ASYNC runs on c->aux and leaves inv_pending set;
// wait_invert joins it (host wait on its event); finish_invert also reports
// a pivot failure it found (CPM_ENOTPD) and publishes s.
cpm_status wait_invert(cpm_ctx* c) {
  if (!c->inv_pending) return CPM_OK;
  c->inv_pending = false;
  HIP_TRY(c, hipEventSynchronize(c->aux_ev));
  c->s_sum = c->h_async->s;
  if (c->h_async->flag != 0) {
    c->pivot = c->h_async->flag - 1;
    c->have_inv = false;
    c->inv_failed = true;
  }
  return CPM_OK;
}

cpm_status finish_invert(cpm_ctx* c) {
  TRY(wait_invert(c));
  if (c->inv_failed) {
    c->inv_failed = false;
    return fail(c, CPM_ENOTPD, "elastance matrix not positive definite at pivot %d", c->pivot);
  }
  return CPM_OK;
}

// ---- kernel timing ---------------------------------------------------------
hipEvent_t take_event(cpm_ctx* c) {
  if (!c->evpool.empty()) {
    hipEvent_t e = c->evpool.back();
    c->evpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// fold finished (or, with wait, all) pending event pairs into the totals
void resolve_timing(cpm_ctx* c, bool wait) {
  std::vector<cpm_ctx::Pending> keep;
  for (auto& p : c->pending) {
    if (!wait && hipEventQuery(p.b) != hipSuccess) {
      keep.push_back(p);
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto& t = c->totals[p.name];
      t.first += ms;
      t.second += 1;
    }
    c->evpool.push_back(p.a);
    c->evpool.push_back(p.b);
  }
  c->pending.swap(keep);
  (void)hipGetLastError();
}

// brackets the launches of one kernel family with events while timing is on
struct Timed {
  cpm_ctx* c;
  const char* name;
  hipStream_t st;
  hipEvent_t a = nullptr;
  Timed(cpm_ctx* c_, const char* n, hipStream_t s_ = nullptr)
      : c(c_), name(n), st(s_ ? s_ : c_->stream) {
    if (!c->timing) return;
    if (!c->timing_only.empty() &&
        std::find(c->timing_only.begin(), c->timing_only.end(), n) == c->timing_only.end())
      return;
    if ((a = take_event(c))) (void)hipEventRecord(a, st);
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) return;
    (void)hipEventRecord(b, st);
    c->pending.push_back({name, a, b});
    if (c->pending.size() > 4096) resolve_timing(c, false);
  }
};

// Half-space k set K+ with |k| <= kc, walked column by column ((nx, ny) with
// nx ascending, then ny ascending) and nz ascending inside a column, cut into
// runs of at most RUN consecutive nz.
void build_kset(cpm_ctx* c, std::vector<KRun>& runs, std::vector<double>& w2,
                std::vector<int>& kx, std::vector<int>& ky, std::vector<int>& kz) {
  const double twopi = 2.0 * M_PI;
  const double Lx = c->p.Lx, Ly = c->p.Ly, Lz = c->Lz, kc = c->kc;
  const int nxm = (int)std::floor(kc * Lx / twopi);
  const int nym = (int)std::floor(kc * Ly / twopi);
  const int nzm = (int)std::floor(kc * Lz / twopi);
  c->nxm = nxm;
  c->nym = nym;
  c->nzm = nzm;
  const double a2 = 4.0 * c->p.alpha * c->p.alpha;
  for (int nx = 0; nx <= nxm; ++nx)
    for (int ny = -nym; ny <= nym; ++ny) {
      if (nx == 0 && ny < 0) continue;
      const int zlo = (nx == 0 && ny == 0) ? 1 : -nzm;
      bool open = false;
      int run_start = 0, cnt = 0;
      for (int nz = zlo; nz <= nzm; ++nz) {
        const double gx = twopi * nx / Lx, gy = twopi * ny / Ly, gz = twopi * nz / Lz;
        const double k2 = gx * gx + gy * gy + gz * gz;
        const bool keep = k2 <= kc * kc;
        if (keep) {
          if (!open || cnt == RUN || nz != run_start + cnt) {
            open = true;
            runs.push_back(KRun{nx, ny, nz, 0, (int)w2.size(), 0});
            run_start = nz;
            cnt = 0;
          }
          w2.push_back(2.0 * (4.0 * M_PI / c->V) * std::exp(-k2 / a2) / k2);
          kx.push_back(nx); ky.push_back(ny); kz.push_back(nz);
          ++cnt;
          runs.back().len = cnt;
        }
      }
    }
}

// charge chunks per configuration for a group of g configurations on the
// matrix-core structure-factor path: about sfm_wg_target workgroups, at most
// sfm_max_chunk charges per chunk (a chunk's table rows, ~1 KB per charge,
// then fit one XCD's L2: large systems), at least sfm_min_chunk (small
// groups: fewer partials to write and sum), and g * chunks a multiple of 8
// (the kernel keeps each (configuration, chunk) pair on one XCD)
int sf_chunks_for(const cpm_ctx* c, int g, bool f16) {
  const int items = f16 ? c->sf16_nitems : c->sfm_nitems;
  const int target = f16 ? c->sf16_wg_target : c->sfm_wg_target;
  const int by_wg = (target + items * g - 1) / (items * g);
  const int by_l2 = (c->m + c->sfm_max_chunk - 1) / c->sfm_max_chunk;
  const int base = std::max(1, std::min(std::max(by_wg, by_l2), c->m / c->sfm_min_chunk));
  int step = 8;
  while (step > 1 && g % (8 / step * 2) == 0) step /= 2;   // step = 8 / gcd(g, 8)
  return (base + step - 1) / step * step;
}

// workgroups of a grouped real-space launch: enough rounds that the planes'
// uneven work evens out (2880 atoms, 64 configurations: 4.3 -> 3.9 us per
// configuration from 512 to 2048; 20064 atoms: 0.81 -> 0.57 ms from 512 to
// 4096), fewer for small atom maps, where every workgroup's staging of the
// pair table costs more than it evens out
int rs_target(const cpm_ctx* c) {
  if (c->rs_wg_target > 0) return c->rs_wg_target;
  const int atom_blocks = (c->nmap + real_space_block_atoms() - 1) / real_space_block_atoms();
  return atom_blocks <= 8 ? 2048 : 4096;
}

// real-space charge chunks for a launch group of g configurations on the
// grouped path: the chunks and the configurations (the grid's third
// dimension) fill about rs_wg_target workgroups together, >= 64 charges per
// chunk
int rchunks_for(const cpm_ctx* c, int g) {
  const int atom_blocks = (c->nmap + real_space_block_atoms() - 1) / real_space_block_atoms();
  const int t = rs_target(c);
  return std::max(1, std::min(std::max(1, c->m / 64), (t + atom_blocks * g - 1) / (atom_blocks * g)));
}

// the planar real-space kernel: atoms on z planes (whole waves per plane in
// the atom map) and at most one periodic image within rc
bool rs_plane(const cpm_ctx* c) {
  const double two_rc = 2.0 * c->p.rcut;
  return c->rs_plane_ok && c->nlayers > 0 && c->p.Lx >= two_rc && c->p.Ly >= two_rc &&
         c->Lz >= two_rc;
}

cpm_status ensure_vat(cpm_ctx* c) {
  return dalloc(c, &c->b.vat, (size_t)c->npad);
}

// slot space of the CG vectors: the atom map for the operator (plane tiles),
// the atoms padded to npad for the dense A
int cg_nslot(const cpm_ctx* c) { return c->have_op ? c->nmap : c->npad; }
const int* cg_slots(const cpm_ctx* c) { return c->have_op ? c->b.amap : c->b.cg_ident; }

// blocks of the CG vector kernels (all share one grid)
// (the partials of one kernel are summed by every workgroup of the next, so
// fewer, fuller workgroups pay off for small operators)
int cg_grid(const cpm_ctx* c) {
  const int cap = c->cg_cap > 0 ? c->cg_cap : std::min(128, std::max(32, cg_nslot(c) / 48));
  return cg_blocks(cg_nslot(c), cap);
}

// AP = A P for the slot-major CG vectors (all CG_MAXG columns): the
// operator's k-space products, then the ELL real space and the rest
// (k_cg_apply); the dense A as one FP64 matrix-core product.  k_cg_apply
// leaves the partials of p.Ap for the step length (partials = true).
void apply_A(cpm_ctx* c, const double* P, double* AP, bool partials) {
  Buffers& b = c->b;
  hipStream_t st = c->stream;
  const int n = c->n, nslot = cg_nslot(c), nblk = cg_grid(c);
  if (c->have_op) {
    { Timed t(c, "cg_plane_sums");
      launch_cg_plane_sums(st, nslot, c->ncp, c->nlayers, c->cg_ksplit, b.plane_off, b.Ecat, P,
                           b.cgY); }
    { Timed t(c, "cg_plane_mix");
      launch_cg_plane_mix(st, c->ncp, c->ncolsort, c->nlayers, c->cg_ksplit, b.Qpair, b.cgY,
                          b.cgT); }
    { Timed t(c, "cg_tiles");
      launch_cg_tiles(st, c->cg_nitems, nslot, c->ncp, b.cg_items, b.Ecat, b.cgT, b.bsr_col,
                      b.bsr_val, P, b.cgphi); }
  } else {
    Timed t(c, "cg_gemm_dense");
    launch_gemm_f64(st, false, false, nslot, CG_MAXG, nslot, 1.0, b.A, c->npad, P, CG_MAXG, 0.0,
                    AP, CG_MAXG, 0, 0);
  }
  if (c->have_op || partials) {
    Timed t(c, "cg_apply");
    launch_cg_apply(st, !c->have_op, nblk, nslot, n, cg_slots(c), b, c->cg_nparts, b.cgphi,
                    c->op_background, c->cdip, c->ke, P, AP, b.cgred);
  }
}

// conjugate-gradient work: X, R, P, AP (slot-major, CG_MAXG columns), block
// partials, scalars, counters; the operator's k-space work arrays
cpm_status ensure_cg_buffers(cpm_ctx* c) {
  Buffers& b = c->b;
  if (b.cgv) return CPM_OK;
  const int nslot = cg_nslot(c);
  if (!c->have_op) {
    std::vector<int> id(c->npad, -1);
    for (int i = 0; i < c->n; ++i) id[i] = i;
    TRY(dalloc(c, &b.cg_ident, id.size()));
    HIP_TRY(c, hipMemcpy(b.cg_ident, id.data(), id.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  TRY(dalloc(c, &b.cgv, (size_t)4 * CG_MAXG * nslot));
  HIP_TRY(c, hipMemset(b.cgv, 0, (size_t)4 * CG_MAXG * nslot * sizeof(double)));
  // partials of the vector kernels' blocks and of the preconditioner's tiles
  const int nred = std::max(cg_grid(c), c->have_op ? nslot / 64 : 0);
  TRY(dalloc(c, &b.cgred, (size_t)nred * CG_RED * CG_MAXG));
  TRY(dalloc(c, &b.cgscal, (size_t)CG_NSCAL * CG_MAXG));
  HIP_TRY(c, hipMemset(b.cgscal, 0, (size_t)CG_NSCAL * CG_MAXG * sizeof(double)));
  if (c->have_op) {
    // parts a tile's work items do not use stay zero
    const size_t phi = (size_t)c->cg_nparts * nslot * CG_MAXG;
    TRY(dalloc(c, &b.cgphi, phi));
    HIP_TRY(c, hipMemset(b.cgphi, 0, phi * sizeof(double)));
    TRY(dalloc(c, &b.cgY, (size_t)c->cg_ksplit * c->nlayers * 2 * c->ncp * CG_MAXG));
    TRY(dalloc(c, &b.cgT, (size_t)c->nlayers * 2 * c->ncp * CG_MAXG));
  }
  return CPM_OK;
}

// The two-level preconditioner of the operator's CG, built on first use:
// inverse diagonal tile blocks B, and the coarse matrix C = Z^T A Z from
// A Z (A applied to the coarse basis vectors, CG_MAXG per application),
// inverted in place; the balancing form also keeps DAZ = B A Z and
// H = C^-1 + C^-1 (A Z)^T DAZ C^-1.  Coarse arrays have row stride ld = the
// coarse-space dimension rounded up to 64 and are zero beyond it.
// Operators with more than PC_MAX_TILES tiles run without a preconditioner.
constexpr int PC_MAX_TILES = 2048;

// a set-up temporary: freed (after the stream has drained) and taken off the
// context's byte count on every return
struct DevTemp {
  cpm_ctx* c;
  double* p = nullptr;
  size_t count = 0;
  explicit DevTemp(cpm_ctx* c_) : c(c_) {}
  cpm_status alloc(size_t n) {
    count = n;
    return dalloc(c, &p, n);
  }
  ~DevTemp() {
    if (!p) return;
    (void)hipStreamSynchronize(c->stream);
    dfree(c, p);
  }
};
// From this many tiles on, the balancing form also takes the in-plane
// offsets into its coarse space: at 20064 atoms (318 tiles) 46 -> 34
// iterations outweigh the threefold coarse products (1580 -> 1720 solves/s);
// at 2880 atoms (48 tiles), 37 -> 29 iterations do not (13.5k -> 13.0k).
constexpr int PC_COARSE3_TILES = 128;

cpm_status ensure_precond(cpm_ctx* c) {
  if (c->pc_ready) return CPM_OK;
  c->pc_tiles = 0;
  c->pc_mode = 0;
  const int nslot = c->nmap, T = nslot / 64;
  if (!c->have_op || c->cg_precond <= 0 || T > PC_MAX_TILES) return CPM_OK;
  const bool bal = c->cg_precond >= 2;
  // basis functions per tile: the constant, and for the balancing form the
  // two in-plane offsets from the tile's centre (scaled by the tile's RMS
  // radius; left out, as zero functions, for tiles with fewer than 8 atoms
  // or a spread more than 10x longer than wide)
  const int kwant = c->pc_k > 0 ? c->pc_k : (T >= PC_COARSE3_TILES ? 3 : 1);
  const int K = bal && (size_t)T * kwant <= 2 * (size_t)PC_MAX_TILES ? kwant : 1;
  const int Tk = T * K, ld = (Tk + 63) / 64 * 64;
  std::vector<double> phi((size_t)nslot * 3, 0.0);
  for (int t = 0; t < T; ++t) {
    std::vector<int> rs;
    for (int r = t * 64; r < t * 64 + 64; ++r)
      if (c->h_amap[r] >= 0) rs.push_back(r);
    for (int r : rs) phi[(size_t)r * 3] = 1.0;
    if (K < 3 || rs.size() < 8) continue;
    const double Lx = c->p.Lx, Ly = c->p.Ly;
    const int i0 = c->h_amap[rs[0]];
    std::vector<double> dx, dy;
    double mx = 0.0, my = 0.0;
    for (int r : rs) {
      const int i = c->h_amap[r];
      double ux = c->h_xyz[3 * i] - c->h_xyz[3 * i0], uy = c->h_xyz[3 * i + 1] - c->h_xyz[3 * i0 + 1];
      ux -= Lx * std::rint(ux / Lx);
      uy -= Ly * std::rint(uy / Ly);
      dx.push_back(ux);
      dy.push_back(uy);
      mx += ux;
      my += uy;
    }
    mx /= rs.size();
    my /= rs.size();
    double sxx = 0.0, syy = 0.0, sxy = 0.0;
    for (size_t q = 0; q < rs.size(); ++q) {
      dx[q] -= mx;
      dy[q] -= my;
      sxx += dx[q] * dx[q];
      syy += dy[q] * dy[q];
      sxy += dx[q] * dy[q];
    }
    const double tr = sxx + syy, det = sxx * syy - sxy * sxy;
    const double disc = std::sqrt(std::max(0.0, 0.25 * tr * tr - det));
    const double lmax = 0.5 * tr + disc, lmin = 0.5 * tr - disc;
    if (!(lmax > 0.0) || lmin < 0.01 * lmax) continue;
    const double h = std::sqrt(tr / rs.size());
    for (size_t q = 0; q < rs.size(); ++q) {
      phi[(size_t)rs[q] * 3 + 1] = dx[q] / h;
      phi[(size_t)rs[q] * 3 + 2] = dy[q] / h;
    }
  }
  Buffers& b = c->b;
  hipStream_t st = c->stream;
  if ((int)c->h_tile_plane.size() != T || (int)c->h_bdiag.size() != T)
    return fail(c, CPM_ESTATE, "operator tiles (%zu planes, %zu blocks) do not match %d slots",
                c->h_tile_plane.size(), c->h_bdiag.size(), nslot);
  const size_t ld2 = (size_t)ld * ld;
  TRY(dalloc(c, &b.pc_dinv, (size_t)T * 4096));
  TRY(dalloc(c, &b.pc_C, ld2));
  TRY(dalloc(c, &b.pc_W, ld2));
  TRY(dalloc(c, &b.pc_ztr, (size_t)ld * CG_MAXG));
  TRY(dalloc(c, &b.pc_phi, phi.size()));
  HIP_TRY(c, hipMemcpyAsync(b.pc_phi, phi.data(), phi.size() * sizeof(double),
                            hipMemcpyHostToDevice, st));
  TRY(dalloc(c, &b.pc_tplane, (size_t)T));
  TRY(dalloc(c, &b.pc_dblk, (size_t)T));
  HIP_TRY(c, hipMemsetAsync(b.pc_C, 0, ld2 * sizeof(double), st));
  HIP_TRY(c, hipMemsetAsync(b.pc_W, 0, ld2 * sizeof(double), st));
  HIP_TRY(c, hipMemsetAsync(b.pc_ztr, 0, (size_t)ld * CG_MAXG * sizeof(double), st));
  HIP_TRY(c, hipMemcpyAsync(b.pc_tplane, c->h_tile_plane.data(), T * sizeof(int),
                            hipMemcpyHostToDevice, st));
  HIP_TRY(c, hipMemcpyAsync(b.pc_dblk, c->h_bdiag.data(), T * sizeof(int), hipMemcpyHostToDevice,
                            st));
  { Timed t(c, "pc_blocks");
    launch_pc_blocks(st, T, nslot, c->nlayers, c->ncolsort, b.amap, b.pc_tplane, b.pc_dblk,
                     b.bsr_val, b.Ecat, b.Qpair, b, c->op_background, c->cdip, c->ke, b.pc_dinv); }
  TRY(launched(c, "preconditioner blocks"));
  double* P = b.cgv + (size_t)2 * CG_MAXG * nslot;
  double* AP = P + (size_t)CG_MAXG * nslot;
  DevTemp azt(c);                         // balancing form: A Z, slots x ld (set-up only)
  double*& AZ = azt.p;
  if (bal) {
    TRY(azt.alloc((size_t)nslot * ld));
    HIP_TRY(c, hipMemsetAsync(AZ, 0, (size_t)nslot * ld * sizeof(double), st));
  }
  const int nb = cg_grid(c);
  { Timed t(c, "pc_coarse_matrix");
    for (int j0 = 0; j0 < Tk; j0 += CG_MAXG) {
      const int g = std::min(CG_MAXG, Tk - j0);
      launch_pc_basis(st, nb, nslot, K, j0, g, b.amap, b.pc_phi, b, P, b.cgred);
      apply_A(c, P, AP, false);
      launch_pc_coarse_cols(st, T, ld, K, j0, g, b.pc_phi, AP, b.pc_C);
      if (bal)
        HIP_TRY(c, hipMemcpy2DAsync(AZ + j0, (size_t)ld * sizeof(double), AP,
                                    CG_MAXG * sizeof(double), (size_t)g * sizeof(double), nslot,
                                    hipMemcpyDeviceToDevice, st));
    }
    c->pc_Cinv = launch_pc_invert(st, Tk, ld, b.pc_C, b.pc_W); }
  TRY(launched(c, "preconditioner coarse matrix"));
  if (bal) {
    Timed t(c, "pc_balancing");
    const int np = std::max(1, std::min(T, 64));
    TRY(dalloc(c, &b.pc_daz, (size_t)nslot * ld));
    TRY(dalloc(c, &b.pc_H, ld2));
    TRY(dalloc(c, &b.pc_ypart, (size_t)np * ld * CG_MAXG));
    TRY(dalloc(c, &b.pc_y, (size_t)ld * CG_MAXG));
    TRY(dalloc(c, &b.pc_wn, (size_t)ld * CG_MAXG));
    TRY(dalloc(c, &b.pc_g, (size_t)ld * CG_MAXG));
    // coarse products split over coarse columns in parts of ~64 once they
    // are long (a single workgroup row would run them serially)
    const int cp = ld >= 256 ? ld / 64 : 1;
    if (cp > 1) TRY(dalloc(c, &b.pc_cpart, (size_t)cp * 2 * ld * CG_MAXG));
    c->pc_cparts = cp;
    DevTemp gmt(c), xt(c);                // (A Z)^T DAZ, and C^-1 times it
    TRY(gmt.alloc(ld2));
    TRY(xt.alloc(ld2));
    double* Gm = gmt.p;
    double* X = xt.p;
    // DAZ: each tile's rows of A Z times that tile's inverse block
    for (int t = 0; t < T; ++t)
      launch_gemm_f64(st, false, false, 64, ld, 64, 1.0, b.pc_dinv + (size_t)t * 4096, 64,
                      AZ + (size_t)t * 64 * ld, ld, 0.0, b.pc_daz + (size_t)t * 64 * ld, ld, 0, 0);
    launch_gemm_f64(st, true, false, ld, ld, nslot, 1.0, AZ, ld, b.pc_daz, ld, 0.0, Gm, ld, 0, 0);
    launch_gemm_f64(st, false, false, ld, ld, ld, 1.0, c->pc_Cinv, ld, Gm, ld, 0.0, X, ld, 0, 0);
    HIP_TRY(c, hipMemcpyAsync(b.pc_H, c->pc_Cinv, ld2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_gemm_f64(st, false, false, ld, ld, ld, 1.0, X, ld, c->pc_Cinv, ld, 1.0, b.pc_H, ld, 0, 0);
    TRY(launched(c, "preconditioner balancing products"));
    HIP_TRY(c, hipStreamSynchronize(st));
    c->pc_nparts = np;
  }
  HIP_TRY(c, hipStreamSynchronize(st));
  c->pc_tiles = T;
  c->pc_ld = ld;
  c->pc_kuse = K;
  c->pc_mode = bal ? 2 : 1;
  c->pc_ready = true;
  return CPM_OK;
}

// z = M^-1 r for the CG group (into Z), with the partials of r.z (parity
// field) and of sum z
void precond_apply(cpm_ctx* c, int parity, const double* R, double* Z) {
  Buffers& b = c->b;
  if (c->pc_mode == 2)
    launch_bnn_apply(c->stream, c->pc_tiles, c->pc_kuse, c->pc_ld, c->pc_nparts, c->pc_cparts,
                     parity, b.amap, b.pc_phi, b.pc_dinv, b.pc_daz, c->pc_Cinv, b.pc_H, R, Z,
                     b.pc_ypart, b.pc_y, b.pc_ztr, b.pc_wn, b.pc_g, b.pc_cpart, b.cgred);
  else
    launch_pc_apply(c->stream, c->pc_tiles, c->pc_ld, parity, b.amap, b.pc_dinv, c->pc_Cinv, R, Z,
                    b.pc_ztr, b.cgred);
}

cpm_status ensure_step_buffers(cpm_ctx* c) {
  Buffers& b = c->b;
  if (c->step_ready) return CPM_OK;
  c->zperm_ok = false;
  // chunking of the per-snapshot sums (fixed per context, so results are
  // reproducible): ~512 workgroups per kernel, >= 64 charges per SF chunk,
  // >= 32 charges per real-space chunk
  const int run_blocks = (c->nruns + 255) / 256;
  const int sf_target = c->sf_wg_target;
  c->mchunks = std::max(1, std::min((sf_target + run_blocks - 1) / run_blocks, std::max(1, c->m / 64)));
  // real space: 2 workgroups per CU fit (pair table in LDS); the charge
  // chunks fill about 512 workgroups together with the configurations of a
  // launch group (the grid's third dimension), so few partials per atom
  // remain (rchunks is set below, once the group size is known)
  const int atom_blocks = (c->nmap + real_space_block_atoms() - 1) / real_space_block_atoms();
  c->rchunks = std::max(1, std::min(512 / atom_blocks, std::max(1, c->m / 32)));
  TRY(dalloc_cap(c, &b.sf_part, (size_t)2 * c->nk * c->mchunks));
  const bool fast = c->sf_mfma && c->nlayers > 0;
  if (c->sf_mfma) {
    c->mpad = std::max(64, (c->m + 63) / 64 * 64);
    // table rows per configuration in double2 units: the FP64 / FP32 layout
    // or the split-FP16 one (float2 rows and the z operand), the larger
    c->sft_rows = std::max(sf_table_rows(c->nxm, c->nym, c->sfm_nbz),
                           (sf16_rows(c->nxm, c->nym, c->sfm_nbz) + 1) / 2);
    c->sft_blocks = (c->mpad + 255) / 256;
    // planar electrodes: configurations per launch group (at most the 64
    // columns of the projection product), within ~1 GB of per-configuration
    // workspace (phase tables, two chunks of structure-factor partials,
    // real-space partials, gathered charges)
    if (fast) {
      const double per = 16.0 * c->sft_rows * c->mpad + 16.0 * c->sfm_pchunk +
                         16.0 * c->n + 32.0 * c->m + 24.0 * ((c->m + 255) / 256);
      c->pv_group = std::max(1, std::min(std::min(CG_MAXG, c->pv_group_cap),
                                         (int)(1024.0 * 1024 * 1024 / per)));
    }
    const int G = c->pv_group;
    size_t part_rows = 0;                 // (configuration, chunk) blocks of sfm_part
    for (int g = 1; g <= G; ++g)
      part_rows = std::max(part_rows, (size_t)g * std::max(sf_chunks_for(c, g, false),
                                                           sf_chunks_for(c, g, true)));
    TRY(dalloc_cap(c, &b.sfm_part, part_rows * c->sfm_pchunk));
    TRY(dalloc_cap(c, &b.sft, (size_t)G * c->sft_rows * c->mpad));
  }
  // (configuration, chunk) rows of the real-space partials
  size_t rrows = (size_t)c->rchunks;
  if (fast)
    for (int g = 1; g <= c->pv_group; ++g) rrows = std::max(rrows, (size_t)g * rchunks_for(c, g));
  TRY(dalloc_cap(c, &b.sfw, (size_t)2 * c->nk));
  const int pk_rows = c->nlayers > 0 ? layer_project_chunks((int)c->h_cols.size()) : c->kchunks;
  TRY(dalloc_cap(c, &b.phik_part, (size_t)c->n * std::max(pk_rows, c->kchunks)));
  TRY(dalloc_cap(c, &b.phir_part, rrows * c->n));
  c->dip_blocks = std::max(1, (c->m + 255) / 256);
  TRY(dalloc_cap(c, &b.dip, (size_t)c->pv_group * c->dip_blocks * 3));
  TRY(dalloc_cap(c, &b.rtab, (size_t)3 * (RS_NT + 1)));
  const size_t mpad64 = (size_t)std::max(64, (c->m + 63) / 64 * 64);
  TRY(dalloc_cap(c, &b.zperm, mpad64));
  TRY(dalloc_cap(c, &b.cq, (size_t)c->pv_group * mpad64));
  TRY(dalloc_cap(c, &b.zr, (size_t)c->pv_group * (mpad64 / 64)));
  launch_pair_table(c->stream, c->p.alpha, c->p.eta, c->p.rcut, b.rtab);
  TRY(launched(c, "pair table"));
  if (!b.ptab) {
    // pair polynomials of the planar real-space kernel: they depend on the
    // context's parameters only, so they are formed once
    std::vector<double> t;
    pair_poly_table(c->p.alpha, c->p.eta, c->p.rcut, t);
    TRY(dalloc(c, &b.ptab, t.size()));
    HIP_TRY(c, hipMemcpy(b.ptab, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  c->step_ready = true;
  return CPM_OK;
}

cpm_status ensure_solve_buffers(cpm_ctx* c, int batch) {
  Buffers& b = c->b;
  if (batch > b.bpad_rows) {
    dfree(c, b.qt); dfree(c, b.res); dfree(c, b.qpad); dfree(c, b.bpad);
    dfree(c, b.xhi); dfree(c, b.xlo);
    const size_t sz = (size_t)batch * c->npad;
    TRY(dalloc(c, &b.qt, sz));
    TRY(dalloc(c, &b.res, sz));
    TRY(dalloc(c, &b.qpad, sz));
    TRY(dalloc(c, &b.bpad, sz));
    TRY(dalloc(c, &b.xhi, sz));
    TRY(dalloc(c, &b.xlo, sz));
    dfree(c, b.means);
    TRY(dalloc(c, &b.means, (size_t)batch));
    // padding rows and columns of these buffers are read by the GEMMs: zero them once
    HIP_TRY(c, hipMemsetAsync(b.qt, 0, sz * sizeof(double), c->stream));
    HIP_TRY(c, hipMemsetAsync(b.res, 0, sz * sizeof(double), c->stream));
    HIP_TRY(c, hipMemsetAsync(b.qpad, 0, sz * sizeof(double), c->stream));
    HIP_TRY(c, hipMemsetAsync(b.bpad, 0, sz * sizeof(double), c->stream));
    b.bpad_rows = batch;
  }
  return CPM_OK;
}

// split-BF16 GEMM configuration for a padded row count: the autotuned one,
// else 64-row tiles, no K split, one workgroup per tile
cpm_ctx::GemmCfg bf16_cfg(const cpm_ctx* c, int rows) {
  auto it = c->tuned.find(rows);
  if (it != c->tuned.end()) return it->second;
  return cpm_ctx::GemmCfg{};
}

cpm_status ensure_kpart(cpm_ctx* c, size_t len) {
  Buffers& b = c->b;
  if (len <= b.kpart_len) return CPM_OK;
  dfree(c, b.kpart);
  TRY(dalloc(c, &b.kpart, len));
  b.kpart_len = len;
  return CPM_OK;
}

// work buffers of one solve: the context's own (grown on demand), or carved
// out of the fixed scratch array of cpm_solve_charges_noalloc
struct SolveWork {
  double* qt; double* res; double* bpad; double* qpad; double* means; double* kpart;
  uint16_t* xhi; uint16_t* xlo;
  const cpm_ctx::GemmCfg* bf16 = nullptr;      // forced split-BF16 configuration
};

SolveWork ctx_work(cpm_ctx* c) {
  Buffers& b = c->b;
  return SolveWork{b.qt, b.res, b.bpad, b.qpad, b.means, b.kpart, b.xhi, b.xlo, nullptr};
}

// one split-BF16 product C (+)= X S~ over `rows` rows of this context; X is
// split into BF16 pairs once, before the product
void enqueue_bf16(cpm_ctx* c, const double* x, double* y, int rows, bool accumulate,
                  const cpm_ctx::GemmCfg& cfg, const SolveWork& w) {
  const int npad = c->npad;
  launch_split_bf16(c->stream, (size_t)rows * npad, x, w.xhi, w.xlo);
  GemmGroupBf grp{};
  grp.nprob = 1;
  grp.p[0] = gemm_bf16x3_problem(rows, npad, npad, w.xhi, w.xlo, npad, c->b.Shi, c->b.Slo,
                                 npad, y, npad, accumulate ? 1 : 0, cfg.bm, cfg.ks, w.kpart);
  group_finish(grp);
  launch_gemm_bf16x3_group(c->stream, grp, cfg.bm, cfg.grid > 0 ? cfg.grid : grp.total);
}

// upload the k set and electrolyte charges on first device use
cpm_status ensure_uploaded(cpm_ctx* c) {
  Buffers& b = c->b;
  if (!b.runs) {
    TRY(dalloc(c, &b.runs, c->h_runs.size()));
    TRY(dalloc(c, &b.w2, c->h_w2.size()));
    TRY(dalloc(c, &b.knx, c->h_kx.size()));
    TRY(dalloc(c, &b.kny, c->h_ky.size()));
    TRY(dalloc(c, &b.knz, c->h_kz.size()));
    TRY(dalloc(c, &b.cols, c->h_cols.size()));
    if (c->sf_mfma) {
      auto up = [&](int** dst, const std::vector<int>& v) -> cpm_status {
        TRY(dalloc(c, dst, v.size()));
        HIP_TRY(c, hipMemcpy(*dst, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice));
        return CPM_OK;
      };
      TRY(up(&b.sc_nx, c->h_sc_nx)); TRY(up(&b.sc_ny, c->h_sc_ny)); TRY(up(&b.sc_lo, c->h_sc_lo));
      TRY(up(&b.sc_len, c->h_sc_len)); TRY(up(&b.sc_koff, c->h_sc_koff)); TRY(up(&b.sc_n0, c->h_sc_n0));
      TRY(up(&b.sc_nidx, c->h_sc_nidx)); TRY(up(&b.tile_nb, c->h_tile_nb));
      TRY(up(&b.tile_off, c->h_tile_off));
      TRY(dalloc(c, &b.sfm_items, c->h_sfm_items.size()));
      HIP_TRY(c, hipMemcpy(b.sfm_items, c->h_sfm_items.data(), c->h_sfm_items.size() * sizeof(int4),
                           hipMemcpyHostToDevice));
      TRY(dalloc(c, &b.sf16_items, c->h_sf16_items.size()));
      HIP_TRY(c, hipMemcpy(b.sf16_items, c->h_sf16_items.data(),
                           c->h_sf16_items.size() * sizeof(int4), hipMemcpyHostToDevice));
    }
    TRY(dalloc(c, &b.chunk_col, c->h_chunk_col.size()));
    TRY(dalloc(c, &b.flag, 4));
    TRY(dalloc(c, &b.scal, 8));
    HIP_TRY(c, hipMemcpy(b.runs, c->h_runs.data(), c->h_runs.size() * sizeof(KRun), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(b.w2, c->h_w2.data(), c->h_w2.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(b.knx, c->h_kx.data(), c->h_kx.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(b.kny, c->h_ky.data(), c->h_ky.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(b.knz, c->h_kz.data(), c->h_kz.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(b.cols, c->h_cols.data(), c->h_cols.size() * sizeof(KCol), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(b.chunk_col, c->h_chunk_col.data(), c->h_chunk_col.size() * sizeof(int),
                         hipMemcpyHostToDevice));
  }
  if (c->have_elyt && !b.elq) {
    TRY(dalloc(c, &b.elq, (size_t)std::max(c->m, 1)));
    if (c->m > 0)
      HIP_TRY(c, hipMemcpy(b.elq, c->h_q.data(), (size_t)c->m * sizeof(double), hipMemcpyHostToDevice));
  }
  return CPM_OK;
}

}  // namespace

extern "C" {

cpm_status cpm_create(const cpm_params* params, void* hip_stream, cpm_ctx** out) {
  if (!out) return CPM_EINVAL;
  *out = nullptr;
  if (!params) return CPM_EINVAL;
  cpm_ctx* c = new (std::nothrow) cpm_ctx();
  if (!c) return CPM_ENOMEM;
  c->p = *params;
  c->stream = static_cast<hipStream_t>(hip_stream);
  const cpm_params& p = c->p;
  cpm_status st = CPM_OK;
  const bool slab = p.geometry == CPM_GEOM_SLAB_EW3DC;
  if (p.geometry != CPM_GEOM_SLAB_EW3DC && p.geometry != CPM_GEOM_WIRE && p.geometry != CPM_GEOM_3D)
    st = fail(c, CPM_EUNSUPPORTED, "geometry %d is not one of slab (0), wire (1), 3D (2)", p.geometry);
  else if (!finite_pos(p.Lx) || !finite_pos(p.Ly) || !finite_pos(p.h))
    st = fail(c, CPM_EINVAL, "Lx, Ly, h must be finite and > 0");
  else if (slab && !(std::isfinite(p.slab_factor) && p.slab_factor > 1.0))
    st = fail(c, CPM_EINVAL, "slab_factor must be > 1");
  else if (!slab && !(std::isfinite(p.slab_factor) && p.slab_factor >= 1.0))
    st = fail(c, CPM_EINVAL, "slab_factor must be >= 1");
  else if (!finite_pos(p.eta) || !finite_pos(p.alpha) || !finite_pos(p.rcut))
    st = fail(c, CPM_EINVAL, "eta, alpha, rcut must be finite and > 0");
  else if (!(p.kcut > 0.0) && !(p.kspace_eps > 0.0 && p.kspace_eps < 1.0))
    st = fail(c, CPM_EINVAL, "need kcut > 0 or 0 < kspace_eps < 1");
  else if (!std::isfinite(p.kcut) || !std::isfinite(p.coulomb_k) || p.coulomb_k < 0.0)
    st = fail(c, CPM_EINVAL, "kcut and coulomb_k must be finite (coulomb_k >= 0)");
  else if (slab && (p.slab_factor - 1.0) * p.h <= p.rcut)
    st = fail(c, CPM_EINVAL, "slab clearance (slab_factor - 1) * h = %g must exceed rcut = %g",
              (p.slab_factor - 1.0) * p.h, p.rcut);
  if (st != CPM_OK) {
    delete c;
    return st;
  }
  c->Lz = p.slab_factor * p.h;
  c->V = p.Lx * p.Ly * c->Lz;
  // dipole term of the boundary geometry, A += k_e sum_d cdip_d r_d r_d^T:
  // slab (x, y periodic, EW3DC in z, Eqs. 10, 12): 4 pi / V on z;
  // wire (z periodic, Eq. 11): 2 pi / V on x and y; 3D periodic (tin foil,
  // the finite-field setting): none
  if (p.geometry == CPM_GEOM_SLAB_EW3DC) c->cdip[2] = 4.0 * M_PI / c->V;
  if (p.geometry == CPM_GEOM_WIRE) c->cdip[0] = c->cdip[1] = 2.0 * M_PI / c->V;
  if (const char* ev = std::getenv("CPM_SF_WG_TARGET")) c->sf_wg_target = std::max(64, std::atoi(ev));
  if (const char* ev = std::getenv("CPM_SFM_WG_TARGET")) c->sfm_wg_target = std::max(8, std::atoi(ev));
  if (const char* ev = std::getenv("CPM_SF16_WG_TARGET")) c->sf16_wg_target = std::max(8, std::atoi(ev));
  if (const char* ev = std::getenv("CPM_SFM_MIN_CHUNK")) c->sfm_min_chunk = std::max(16, std::atoi(ev));
  if (const char* ev = std::getenv("CPM_SFM_MAX_CHUNK")) c->sfm_max_chunk = std::max(64, std::atoi(ev));
  if (const char* ev = std::getenv("CPM_RS_WG_TARGET")) c->rs_wg_target = std::max(8, std::atoi(ev));
  if (const char* ev = std::getenv("CPM_RS_SORT_MIN")) c->rs_sort_min = std::max(1, std::atoi(ev));
  if (const char* ev = std::getenv("CPM_PV_FAST_MIN")) c->pv_fast_min = std::max(1, std::atoi(ev));
  if (const char* ev = std::getenv("CPM_PV_GROUP")) c->pv_group_cap = std::max(1, std::atoi(ev));
  if (const char* ev = std::getenv("CPM_RS_CONCURRENT")) c->rs_conc_ok = std::atoi(ev) != 0;
  if (const char* ev = std::getenv("CPM_CG_BLOCKS")) c->cg_cap = std::max(1, std::atoi(ev));
  if (const char* ev = std::getenv("CPM_CG_COARSE")) c->pc_k = std::atoi(ev) >= 3 ? 3 : 1;
  if (const char* ev = std::getenv("CPM_CG_GRAPH")) c->cg_graphs = std::atoi(ev) != 0;
  if (const char* ev = std::getenv("CPM_CG_PRECOND")) c->cg_precond = std::max(0, std::min(2, std::atoi(ev)));
  if (const char* ev = std::getenv("CPM_CHOL_BLOCK"))
    c->chol_block = std::max(1, std::min(32, std::atoi(ev) / TILE)) * TILE;
  if (const char* ev = std::getenv("CPM_SF_MFMA")) c->use_sf_mfma = std::atoi(ev) != 0;
  if (const char* ev = std::getenv("CPM_SF_FP32")) c->sf32_ok = std::atoi(ev) != 0;
  if (const char* ev = std::getenv("CPM_SF_F16")) c->sf16_ok = std::atoi(ev) != 0;
  if (const char* ev = std::getenv("CPM_SF16_NT")) {
    const int v = std::atoi(ev);
    c->sf16_nt = v >= 4 ? 4 : v >= 2 ? 2 : 1;
  }
  if (const char* ev = std::getenv("CPM_RS_PLANE")) c->rs_plane_ok = std::atoi(ev) != 0;
  c->kc = (p.kcut > 0.0) ? p.kcut : 2.0 * p.alpha * std::sqrt(std::log(1.0 / p.kspace_eps));
  c->ke = (p.coulomb_k > 0.0) ? p.coulomb_k : KE_DEFAULT;

  build_kset(c, c->h_runs, c->h_w2, c->h_kx, c->h_ky, c->h_kz);
  c->nk = (int)c->h_w2.size();
  c->nruns = (int)c->h_runs.size();
  if (c->nk == 0) {
    delete c;
    return CPM_EINVAL;
  }
  // projection: column segments (consecutive runs of one (nx, ny), at most
  // PJ_MAXK k values) grouped greedily into chunks of at most PJ_MAXK k values
  for (const KRun& r : c->h_runs) {
    if (!c->h_cols.empty()) {
      KCol& last = c->h_cols.back();
      if (last.nx == r.nx && last.ny == r.ny && last.lo + last.len == r.nz0 &&
          last.len + r.len <= PJ_MAXK) {
        last.len += r.len;
        continue;
      }
    }
    c->h_cols.push_back(KCol{r.nx, r.ny, r.nz0, r.len, r.koff, 0});
  }
  c->h_chunk_col.push_back(0);
  int acc = 0;
  for (int k = 0; k < (int)c->h_cols.size(); ++k) {
    if (acc + c->h_cols[k].len > PJ_MAXK) {
      c->h_chunk_col.push_back(k);
      acc = 0;
    }
    acc += c->h_cols[k].len;
  }
  c->h_chunk_col.push_back((int)c->h_cols.size());
  c->kchunks = (int)c->h_chunk_col.size() - 1;
  // matrix-core structure factors: whole columns, sorted by k_z extent e = max |n|
  {
    struct FC { int nx, ny, lo, len, koff, e; };
    std::vector<FC> fc;
    for (const KRun& r : c->h_runs) {
      if (!fc.empty() && fc.back().nx == r.nx && fc.back().ny == r.ny &&
          fc.back().lo + fc.back().len == r.nz0) {
        fc.back().len += r.len;
      } else {
        fc.push_back(FC{r.nx, r.ny, r.nz0, r.len, r.koff, 0});
      }
    }
    int emax = 0;
    for (FC& f : fc) {
      f.e = std::max(std::abs(f.lo), std::abs(f.lo + f.len - 1));
      emax = std::max(emax, f.e);
    }
    std::stable_sort(fc.begin(), fc.end(), [](const FC& a, const FC& b) { return a.e > b.e; });
    c->ncolsort = (int)fc.size();
    c->sfm_tiles = (c->ncolsort + 15) / 16;
    int nbmax = 0;
    c->h_sc_nidx.push_back(0);
    for (int k = 0; k < c->ncolsort; ++k) {
      const FC& f = fc[k];
      c->h_sc_nx.push_back(f.nx); c->h_sc_ny.push_back(f.ny); c->h_sc_lo.push_back(f.lo);
      c->h_sc_len.push_back(f.len); c->h_sc_koff.push_back(f.koff); c->h_sc_n0.push_back(0);
      c->h_sc_nidx.push_back(c->h_sc_nidx.back() + f.e + 1);
      if (k % 16 == 0) {
        const int nb = (2 * (f.e + 1) + 15) / 16;   // first column of a tile has its largest extent
        c->h_tile_nb.push_back(nb);
        nbmax = std::max(nbmax, nb);
      }
    }
    c->sfm_ntot = c->h_sc_nidx.back();
    c->sfm_npadc = 16 * nbmax;
    c->sfm_nbz = std::max(2, nbmax);           // Z8 rows: first block of every item, and e^{2 pi i 8 fz}
    // work items: each M tile's n blocks split evenly into parts of <= SFM_NB
    for (int mt = 0; mt < c->sfm_tiles; ++mt) {
      const int nb = c->h_tile_nb[mt];
      const int parts = (nb + SFM_NB - 1) / SFM_NB;
      for (int q = 0; q < parts; ++q) {
        const int lo = nb * q / parts, hi = nb * (q + 1) / parts;
        c->h_sfm_items.push_back(make_int4(mt, lo, hi - lo, 0));
      }
    }
    // split-FP16 items: sf16_nt M tiles (mt, mt + 1, ..; tile extents do not
    // grow with mt, so mt's blocks cover them all), blocks in parts of
    // <= SF16_NB (<= 8 with four tiles)
    const int nt16 = c->sf16_nt, nbmax16 = nt16 == 4 ? 8 : SF16_NB;
    for (int mt = 0; mt < c->sfm_tiles; mt += nt16) {
      const int nb = c->h_tile_nb[mt];
      const int nt = std::min(nt16, c->sfm_tiles - mt);
      const int parts = (nb + nbmax16 - 1) / nbmax16;
      for (int q = 0; q < parts; ++q) {
        const int lo = nb * q / parts, hi = nb * (q + 1) / parts;
        c->h_sf16_items.push_back(make_int4(mt, lo, hi - lo, nt));
      }
    }
    c->sf16_nitems = (int)c->h_sf16_items.size();
    c->sfm_nitems = (int)c->h_sfm_items.size();
    c->sf_mfma = c->sfm_nitems > 0;
    // compact partial layout: tile mt holds a 32 x 16 nb_mt block
    int off = 0;
    for (int mt = 0; mt < c->sfm_tiles; ++mt) {
      c->h_tile_off.push_back(off);
      off += 32 * 16 * c->h_tile_nb[mt];
    }
    c->sfm_pchunk = off;
    for (int k = 0; k < c->ncolsort; ++k)
      c->sfm_maxcnt = std::max(c->sfm_maxcnt, c->h_sc_nidx[k + 1] - c->h_sc_nidx[k]);
    (void)emax;
  }
  *out = c;
  return CPM_OK;
}

cpm_status cpm_set_electrolyte(cpm_ctx* c, int m, const double* h_q) {
  if (!c) return CPM_EINVAL;
  if (m < 0 || (m > 0 && !h_q)) return fail(c, CPM_EINVAL, "m must be >= 0 and h_q non-NULL");
  double sum = 0.0, asum = 0.0;
  for (int j = 0; j < m; ++j) {
    if (!std::isfinite(h_q[j])) return fail(c, CPM_EINVAL, "electrolyte charge %d not finite", j);
    sum += h_q[j];
    asum += std::fabs(h_q[j]);
  }
  if (std::fabs(sum) > 1e-10 * std::max(asum, 1e-300) && m > 0)
    return fail(c, CPM_EINVAL, "electrolyte not neutral: sum q = %g", sum);
  if (c->have_elyt) return fail(c, CPM_ESTATE, "electrolyte already set for this context");
  c->m = m;
  c->h_q.assign(h_q, h_q + m);
  c->have_elyt = true;
  return CPM_OK;
}

}  // extern "C"

namespace {

// Enqueue the assembly of the dense elastance A on stream st (Eq. 2 with
// the Ewald split; lower triangle, then mirrored) for the electrodes of the
// last cpm_build_elastance.  Reads only context-owned buffers.
cpm_status assemble_A(cpm_ctx* c, hipStream_t st) {
  if (!c->A_pending) return CPM_OK;
  c->A_pending = false;
  const cpm_params& p = c->p;
  const int n = c->n, npad = c->npad;
  Buffers& b = c->b;
  const double eta_ee = p.eta / std::sqrt(2.0);
  const double diag_self = (std::sqrt(2.0) * p.eta - 2.0 * p.alpha) / std::sqrt(M_PI);
  const double background = -M_PI / (c->V * p.alpha * p.alpha);
  { Timed t(c, "assemble_real", st);
    launch_real_space_A(st, n, npad, b, p.Lx, p.Ly, c->Lz, p.rcut, p.alpha, eta_ee,
                        diag_self, background, c->cdip, c->ke, c->A_diag_extra ? b.dextra : nullptr, b.A); }
  TRY(launched(c, "real_space_A"));
  if (c->nlayers > 0 && c->sf_mfma) {
    // planar electrodes: per plane, A[rows of L] += k_e G_L F^L (K = 2 x columns);
    // Q, G and F stay allocated for rebuilds of the same context
    Timed t(c, "assemble_kspace", st);
    const int ldG = (2 * c->ncolsort + 15) / 16 * 16;
    TRY(dalloc(c, &b.Qpair, (size_t)c->ncolsort * c->nlayers * c->nlayers));
    TRY(dalloc(c, &b.asmG, (size_t)c->nmap * ldG));
    TRY(dalloc(c, &b.asmF, (size_t)ldG * npad));
    launch_plane_pair_weights(st, c->ncolsort, c->nlayers, b.sc_lo, b.sc_len, b.sc_koff,
                              b.w2, b.layer_fz, b.Qpair);
    launch_build_G(st, c->nmap, c->ncolsort, ldG, b.amap, b.sc_nx, b.sc_ny, b, b.asmG);
    int row0 = 0;
    for (int L = 0; L < c->nlayers; ++L) {
      const int rows = c->h_plane_rows[L];              // this plane's rows of the map (x 64)
      // only the lower triangle of A is kept (mirrored at the end): the
      // plane's rows need the columns up to their largest atom index
      int amax = 0;
      for (int r = row0; r < row0 + rows; ++r) amax = std::max(amax, c->h_amap[r]);
      const int ncols = std::min(npad, (amax + 64) / 64 * 64);
      launch_build_F(st, L, n, npad, c->nlayers, c->ncolsort, ldG, b.sc_nx, b.sc_ny, b,
                     b.Qpair, b.asmF);
      launch_gemm_f64(st, false, false, rows, ncols, ldG, c->ke, b.asmG + (size_t)row0 * ldG,
                      ldG, b.asmF, npad, 1.0, b.A, npad, 0, 0, b.amap + row0);
      TRY(launched(c, "kspace planes"));
      row0 += rows;
    }
  } else {
    // k space: A += T T^T over chunks of KC k-vectors (2 KC columns)
    const int KC = 2048;
    TRY(dalloc(c, &b.table, (size_t)npad * 2 * KC));
    for (int k0 = 0; k0 < c->nk; k0 += KC) {
      launch_phase_table(st, n, npad, k0, KC, c->nk, b, c->ke, b.table);
      launch_gemm_f64(st, false, true, npad, npad, 2 * KC, 1.0, b.table, 2 * KC, b.table,
                      2 * KC, 1.0, b.A, npad, /*tri=*/1, 0);
      TRY(launched(c, "kspace syrk"));
    }
    HIP_TRY(c, hipStreamSynchronize(st));
    dfree(c, b.table);
  }
  launch_mirror_lower(st, npad, b.A);
  TRY(launched(c, "mirror"));
  return CPM_OK;
}

// 64-bit FNV-1a over a byte range, continuing from h
uint64_t fnv1a(uint64_t h, const void* data, size_t len) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < len; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Fingerprint of the elastance's inputs: the method knobs (as resolved), the
// electrode coordinates and ids as given, and the diagonal term.
uint64_t geometry_hash(const cpm_ctx* c, int n, int n_e, const double* xyz, const int* eid,
                       const double* diag_extra) {
  uint64_t h = 1469598103934665603ull;
  const cpm_params& p = c->p;
  const double knobs[12] = {p.Lx, p.Ly, p.h, p.slab_factor, p.eta, p.alpha, p.rcut,
                            p.kspace_eps, p.kcut, c->ke, c->Lz, c->kc};
  h = fnv1a(h, knobs, sizeof knobs);
  const int ints[4] = {p.geometry, n, n_e, diag_extra ? 1 : 0};
  h = fnv1a(h, ints, sizeof ints);
  h = fnv1a(h, xyz, (size_t)3 * n * sizeof(double));
  h = fnv1a(h, eid, (size_t)n * sizeof(int));
  if (diag_extra) h = fnv1a(h, diag_extra, (size_t)n * sizeof(double));
  return h;
}

// A^-1, S, u, d, v, the cached response S G and the reduced-precision
// copies of S named by store_flags
cpm_status ensure_inverse_buffers(cpm_ctx* c, unsigned store_flags, bool factor = false) {
  Buffers& b = c->b;
  const int npad = c->npad;
  if (factor) {
    TRY(dalloc(c, &b.u, npad));
    TRY(dalloc(c, &b.d, npad));
    TRY(dalloc(c, &b.vat, npad));
    TRY(dalloc_cap(c, &b.sg, (size_t)npad * c->n_e));
    TRY(dalloc_cap(c, &b.fwork, (size_t)2 * TILE * npad));
    return CPM_OK;
  }
  TRY(dalloc(c, &b.Ainv, (size_t)npad * npad));
  TRY(dalloc(c, &b.S, (size_t)npad * npad));
  TRY(dalloc(c, &b.u, npad));
  TRY(dalloc(c, &b.d, npad));
  TRY(dalloc(c, &b.vat, npad));
  if (c->n_e <= CCM_MAXE) TRY(dalloc_cap(c, &b.sg, (size_t)npad * c->n_e));
  if (store_flags & CPM_STORE_F32) TRY(dalloc(c, &b.S32, (size_t)npad * npad));
  if (store_flags & CPM_STORE_BF16X2) {
    TRY(dalloc(c, &b.Shi, (size_t)npad * npad));
    TRY(dalloc(c, &b.Slo, (size_t)npad * npad));
  }
  return CPM_OK;
}

// X <- X A^-1 for `rows` right-hand sides stored as rows (stride npad,
// rows a multiple of 64) with the Cholesky factor A = L L^T (b.L, lower;
// b.Dinv the inverses of its 64 x 64 diagonal blocks): Y L^T = X by blocks
// left to right, then Z L = Y right to left, Z into X (Y: work of the same
// shape).  Each block step is two MFMA GEMMs: the block times its diagonal
// inverse, then the update of the blocks still to come with one panel of L.
// 2 rows n^2 flop per direction; every sum in a fixed order.
cpm_status factor_solve_rows(cpm_ctx* c, hipStream_t st, int rows, double* X, double* Y) {
  const int npad = c->npad, nb = npad / TILE;
  const Buffers& b = c->b;
  Timed t(c, "factor_solve", st);
  for (int k = 0; k < nb; ++k) {
    const int c0 = k * TILE, rest = npad - c0 - TILE;
    const double* Dk = b.Dinv + (size_t)k * TILE * TILE;
    launch_gemm_f64(st, false, true, rows, TILE, TILE, 1.0, X + c0, npad, Dk, TILE, 0.0, Y + c0,
                    npad, 0, 0);
    if (rest > 0)
      launch_gemm_f64(st, false, true, rows, rest, TILE, -1.0, Y + c0, npad,
                      b.L + (size_t)(c0 + TILE) * npad + c0, npad, 1.0, X + c0 + TILE, npad, 0, 0);
  }
  for (int k = nb - 1; k >= 0; --k) {
    const int c0 = k * TILE;
    const double* Dk = b.Dinv + (size_t)k * TILE * TILE;
    launch_gemm_f64(st, false, false, rows, TILE, TILE, 1.0, Y + c0, npad, Dk, TILE, 0.0, X + c0,
                    npad, 0, 0);
    if (c0 > 0)
      launch_gemm_f64(st, false, false, rows, c0, TILE, -1.0, X + c0, npad, b.L + (size_t)c0 * npad,
                      npad, 1.0, Y, npad, 0, 0);
  }
  return launched(c, "factor solve");
}

// factor-only inverse: u = A^-1 e, s = e^T u and the response S G (Eqs. 4,
// 6) from the solves with the electrode indicators
cpm_status factor_response(cpm_ctx* c, hipStream_t st) {
  Buffers& b = c->b;
  const int npad = c->npad;
  double* X = b.fwork;
  double* Y = b.fwork + (size_t)TILE * npad;
  launch_group_indicator(st, c->n, npad, TILE, b.eid, c->n_e, X);
  TRY(factor_solve_rows(c, st, TILE, X, Y));
  launch_factor_response(st, c->n, npad, c->n_e, X, npad, b.u, b.scal, b.sg);
  c->szeta_ok = false;
  c->have_q = false;
  return launched(c, "factor response");
}

// y = S x for one vector (npad, padding zero): one pass over S, or with the
// factor-only inverse x A^-1 by substitution and the projection P
cpm_status apply_S_one(cpm_ctx* c, const double* x, double* y) {
  if (!c->factor_only) {
    launch_matvec(c->stream, 0, c->npad, c->b.S, 1, x, nullptr, 0, 0.0, y, c->npad, 0);
    return launched(c, "S x");
  }
  Buffers& b = c->b;
  const int npad = c->npad;
  double* X = b.fwork;
  double* Y = b.fwork + (size_t)TILE * npad;
  launch_pad_rows(c->stream, npad, npad, 1, TILE, x, 0, nullptr, X);
  TRY(factor_solve_rows(c, c->stream, TILE, X, Y));
  launch_finalize(c->stream, c->n, 1, X, npad, nullptr, b.u, b.scal, b.eid, c->n_e, y, npad,
                  nullptr);
  return launched(c, "S x (factor)");
}

// From A^-1 in b.Ainv: u = A^-1 e, s = e^T u, S = A^-1 - u u^T / s (Eq. 4),
// the response S G (Eq. 6) and the copies of S named by store_flags, on st.
cpm_status form_S(cpm_ctx* c, hipStream_t st, unsigned store_flags) {
  Buffers& b = c->b;
  const int n = c->n, npad = c->npad;
  HIP_TRY(c, hipMemsetAsync(b.u, 0, npad * sizeof(double), st));
  { Timed t(c, "make_S", st);
    launch_row_sums(st, n, npad, b.Ainv, b.u);
    launch_sum_vector(st, n, b.u, b.scal);
    launch_make_S(st, n, npad, b.Ainv, b.u, b.scal, b.S); }
  TRY(launched(c, "projection"));
  // the response of the charges to each electrode's potential, S G (Eq. 6):
  // a new v~ then costs O(n n_e) instead of a pass over S
  if (b.sg) {
    Timed t(c, "response_SG", st);
    launch_ccm_response(st, n, npad, b.S, b.eid, c->n_e, b.sg);
  }
  TRY(launched(c, "response"));
  c->szeta_ok = false;
  if (store_flags & (CPM_STORE_F32 | CPM_STORE_BF16X2)) {
    Timed t(c, "convert_S", st);
    launch_convert_S(st, npad, b.S, (store_flags & CPM_STORE_F32) ? b.S32 : nullptr,
                     (store_flags & CPM_STORE_BF16X2) ? b.Shi : nullptr,
                     (store_flags & CPM_STORE_BF16X2) ? b.Slo : nullptr);
  }
  TRY(launched(c, "convert"));
  c->store = store_flags | CPM_STORE_F64;
  c->have_q = false;                     // charge targets refer to the previous inverse
  return CPM_OK;
}

// Electrode set-up shared by the dense elastance (dense = true: assemble A)
// and the matrix-free operator (dense = false: keep what A x needs).
cpm_status build_impl(cpm_ctx* c, int n, const double* d_xyz, const int* d_eid, int n_e,
                      const double* d_diag_extra, bool dense) {
  TRY(wait_invert(c));                    // the pending inversion still reads A
  c->inv_failed = false;
  if (n <= 0 || n_e <= 0 || !d_xyz || !d_eid)
    return fail(c, CPM_EINVAL, "need n > 0, n_e > 0 and non-NULL coordinates and ids");
  if ((c->have_A || c->have_op) && n != c->n)
    return fail(c, CPM_EINVAL, "rebuild with n = %d differs from n = %d of this context", n, c->n);
  if ((dense && c->have_op) || (!dense && c->have_A))
    return fail(c, CPM_ESTATE, "a context holds either the dense elastance or the operator");
  TRY(ensure_uploaded(c));
  c->h_xyz.resize((size_t)3 * n);
  c->h_eid.resize(n);
  HIP_TRY(c, hipMemcpy(c->h_xyz.data(), d_xyz, (size_t)3 * n * sizeof(double), hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(c->h_eid.data(), d_eid, (size_t)n * sizeof(int), hipMemcpyDeviceToHost));
  double zmin = 1e300, zmax = -1e300;
  for (int i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(c->h_xyz[3 * i + a])) return fail(c, CPM_EINVAL, "coordinate of atom %d not finite", i);
    if (c->h_eid[i] < 0 || c->h_eid[i] >= n_e)
      return fail(c, CPM_EINVAL, "electrode id %d of atom %d outside [0, %d)", c->h_eid[i], i, n_e);
    zmin = std::min(zmin, c->h_xyz[3 * i + 2]);
    zmax = std::max(zmax, c->h_xyz[3 * i + 2]);
  }
  if (c->p.geometry == CPM_GEOM_SLAB_EW3DC && c->Lz - (zmax - zmin) <= c->p.rcut)
    return fail(c, CPM_EINVAL, "electrode z extent %g leaves no slab clearance in Lz = %g", zmax - zmin, c->Lz);
  {
    // fingerprint of everything A depends on, checked by cpm_load
    std::vector<double> dx;
    if (d_diag_extra) {
      dx.resize(n);
      HIP_TRY(c, hipMemcpy(dx.data(), d_diag_extra, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
    }
    c->geom_hash = geometry_hash(c, n, n_e, c->h_xyz.data(), c->h_eid.data(),
                                 d_diag_extra ? dx.data() : nullptr);
  }
  // planar electrodes: atoms sharing an exact z value form a plane
  std::vector<double> zs;
  for (int i = 0; i < n; ++i) zs.push_back(c->h_xyz[3 * i + 2]);
  std::sort(zs.begin(), zs.end());
  zs.erase(std::unique(zs.begin(), zs.end()), zs.end());
  const int nlayers = (int)zs.size() <= MAX_LAYERS ? (int)zs.size() : 0;
  if ((c->have_A || c->have_op) && (nlayers != c->nlayers))
    return fail(c, CPM_EINVAL, "rebuild changes the electrode plane structure; create a new context");
  if (!dense && !(nlayers > 0 && c->sf_mfma))
    return fail(c, CPM_EUNSUPPORTED, "the matrix-free operator needs electrodes on z planes");
  Buffers& b0 = c->b;
  HIP_TRY(c, hipStreamSynchronize(c->stream));   // queued work may still use what is freed
  c->have_A = c->have_op = c->have_inv = c->have_v = c->have_q = false;
  // the b-path work arrays follow the sizes of the atom map and of the
  // k-set (chunks, launch groups): sized again on first use, keeping
  // allocations that are large enough
  c->step_ready = false;
  // the CG work arrays and the preconditioner follow the atom map and the
  // operator (slots, chunks, work parts): a rebuild allocates them afresh
  dfree(c, b0.cg_ident); dfree(c, b0.cgv); dfree(c, b0.cgred); dfree(c, b0.cgscal);
  dfree(c, b0.cgphi); dfree(c, b0.cgY); dfree(c, b0.cgT);
  dfree(c, b0.pc_phi); dfree(c, b0.pc_dinv); dfree(c, b0.pc_C); dfree(c, b0.pc_W); dfree(c, b0.pc_ztr);
  dfree(c, b0.pc_tplane); dfree(c, b0.pc_dblk); dfree(c, b0.pc_daz); dfree(c, b0.pc_H);
  dfree(c, b0.pc_ypart); dfree(c, b0.pc_y); dfree(c, b0.pc_wn); dfree(c, b0.pc_g);
  dfree(c, b0.pc_cpart);
  // constrained charges and the cached responses S G follow n_e (and A)
  dfree(c, b0.ccmU); dfree(c, b0.ccmC);
  if (n_e > CCM_MAXE) dfree(c, b0.sg);   // else resized by the next inversion
  dfree(c, b0.zeta); dfree(c, b0.szeta);
  c->szeta_ok = false;
  c->pc_ready = false;
  c->pc_tiles = 0;
  c->pc_Cinv = nullptr;
  c->nlayers = nlayers;
  c->n = n;
  c->n_e = n_e;
  c->npad = ((n + TILE - 1) / TILE) * TILE;
  const int npad = c->npad;
  Buffers& b = c->b;
  TRY(dalloc(c, &b.ex, n)); TRY(dalloc(c, &b.ey, n)); TRY(dalloc(c, &b.ez, n));
  TRY(dalloc(c, &b.efx, n)); TRY(dalloc(c, &b.efy, n)); TRY(dalloc(c, &b.efz, n));
  TRY(dalloc(c, &b.eid, n));
  if (dense) TRY(dalloc(c, &b.A, (size_t)npad * npad));
  if (c->nlayers > 0) {
    std::vector<int> lay(n);
    std::vector<double> lfz(c->nlayers);
    for (int L = 0; L < c->nlayers; ++L) lfz[L] = zs[L] / c->Lz;
    for (int i = 0; i < n; ++i)
      lay[i] = (int)(std::lower_bound(zs.begin(), zs.end(), c->h_xyz[3 * i + 2]) - zs.begin());
    TRY(dalloc(c, &b.layer_of, n));
    TRY(dalloc(c, &b.layer_fz, c->nlayers));
    TRY(dalloc(c, &b.layerT, c->h_cols.size() * (size_t)c->nlayers));
    HIP_TRY(c, hipMemcpy(b.layer_of, lay.data(), n * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(b.layer_fz, lfz.data(), c->nlayers * sizeof(double), hipMemcpyHostToDevice));
  }
  {
    // real-space thread map: the atoms of each z plane fill whole waves
    // (non-planar electrodes: caller order); -1 pads each group to 64
    std::vector<int> amap;
    if (c->nlayers > 0) {
      std::vector<std::vector<int>> per(c->nlayers);
      for (int i = 0; i < n; ++i)
        per[std::lower_bound(zs.begin(), zs.end(), c->h_xyz[3 * i + 2]) - zs.begin()].push_back(i);
      c->h_plane_rows.clear();
      for (auto& v : per) {
        // spatially compact 64-atom tiles: serpentine strips along x about
        // one tile (64 atoms at the plane's density) wide, y within a strip
        // (only the order inside the plane changes; every sum over an atom's
        // partners keeps its own fixed order)
        const double Lx = c->p.Lx, Ly = c->p.Ly;
        const double side = std::sqrt(64.0 * Lx * Ly / std::max<size_t>(v.size(), 1));
        const int nb = std::max(1, (int)std::lround(Lx / side));
        auto key = [&](int i) {
          const double x = c->h_xyz[3 * i] - Lx * std::floor(c->h_xyz[3 * i] / Lx);
          const double y = c->h_xyz[3 * i + 1] - Ly * std::floor(c->h_xyz[3 * i + 1] / Ly);
          const int bx = std::min(nb - 1, (int)(x / (Lx / nb)));
          return std::make_pair(bx, (bx & 1) ? -y : y);
        };
        std::stable_sort(v.begin(), v.end(), [&](int a, int b2) { return key(a) < key(b2); });
        const size_t before = amap.size();
        amap.insert(amap.end(), v.begin(), v.end());
        while (amap.size() % 64) amap.push_back(-1);
        c->h_plane_rows.push_back((int)(amap.size() - before));
      }
    } else {
      for (int i = 0; i < n; ++i) amap.push_back(i);
      while (amap.size() % 64) amap.push_back(-1);
    }
    if (b.amap && (int)amap.size() != c->nmap) dfree(c, b.amap);
    c->nmap = (int)amap.size();
    c->h_amap = amap;
    TRY(dalloc(c, &b.amap, amap.size()));
    HIP_TRY(c, hipMemcpy(b.amap, amap.data(), amap.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  HIP_TRY(c, hipMemcpyAsync(b.eid, d_eid, (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
  const cpm_params& p = c->p;
  launch_prep_electrodes(c->stream, n, d_xyz, p.Lx, p.Ly, c->Lz, b);
  TRY(launched(c, "prep_electrodes"));
  if (c->nlayers > 0 && c->sf_mfma) {
    // fixed data of the planar k-space products: plane phases, the in-plane
    // phases as a real (2 ncp) x slots matrix in atom-map order, the atom ->
    // slot map, and the work items of the b-path projection
    const int nzt = c->sfm_npadc / 2, nslot = c->nmap, T = nslot / 64;
    TRY(dalloc(c, &b.pz, (size_t)c->nlayers * nzt));
    launch_plane_phases(c->stream, c->nlayers, nzt, b.layer_fz, b.pz);
    c->ncp = (c->ncolsort + 31) / 32 * 32;
    c->h_tile_plane.clear();
    for (int L = 0; L < c->nlayers; ++L)
      for (int t = 0; t < c->h_plane_rows[L] / 64; ++t) c->h_tile_plane.push_back(L);
    const int kunits = 2 * c->ncp / 64;
    const int u = std::max(2, (T * kunits + 511) / 512);
    const int nk = (kunits + u - 1) / u;           // projection parts per slot tile
    std::vector<int> items, slot_of(n, -1);
    for (int I = 0; I < T; ++I)
      for (int q = 0; q < nk; ++q)
        items.insert(items.end(), {I, 0, kunits * q / nk * 64, kunits * (q + 1) / nk * 64, q,
                                   c->h_tile_plane[I]});
    for (int r = 0; r < nslot; ++r)
      if (c->h_amap[r] >= 0) slot_of[c->h_amap[r]] = r;
    if (c->planar_nslot != nslot || c->b_nparts != nk) {   // sizes follow the atom map
      dfree(c, b.Ecat); dfree(c, b.slot_of); dfree(c, b.b_items); dfree(c, b.bT);
      dfree(c, b.bPhi);
    }
    c->planar_nslot = nslot;
    c->b_nitems = T * nk;
    c->b_nparts = nk;
    TRY(dalloc(c, &b.Ecat, (size_t)2 * c->ncp * nslot));
    TRY(dalloc(c, &b.slot_of, (size_t)n));
    TRY(dalloc(c, &b.b_items, items.size()));
    if (!b.bT) {
      TRY(dalloc(c, &b.bT, (size_t)c->nlayers * 2 * c->ncp * CG_MAXG));
      HIP_TRY(c, hipMemset(b.bT, 0, (size_t)c->nlayers * 2 * c->ncp * CG_MAXG * sizeof(double)));
    }
    TRY(dalloc(c, &b.bPhi, (size_t)nk * nslot * CG_MAXG));
    HIP_TRY(c, hipMemcpy(b.slot_of, slot_of.data(), n * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(b.b_items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice));
    launch_cg_ephase(c->stream, nslot, c->ncp, c->ncolsort, b.amap, b, b.Ecat);
    TRY(launched(c, "planar phases"));
  }
  const double eta_ee = p.eta / std::sqrt(2.0);
  const double diag_self = (std::sqrt(2.0) * p.eta - 2.0 * p.alpha) / std::sqrt(M_PI);
  const double background = -M_PI / (c->V * p.alpha * p.alpha);
  if (!dense) {
    // matrix-free A x: plane-pair weights Q, plane offsets in the atom map,
    // the real-space + self part as a sparse ELL matrix, the diagonal extra
    TRY(dalloc(c, &b.Qpair, (size_t)c->ncolsort * c->nlayers * c->nlayers));
    launch_plane_pair_weights(c->stream, c->ncolsort, c->nlayers, b.sc_lo, b.sc_len, b.sc_koff,
                              b.w2, b.layer_fz, b.Qpair);
    std::vector<int> poff(c->nlayers + 1, 0);
    const std::vector<int>& tplane = c->h_tile_plane;
    for (int L = 0; L < c->nlayers; ++L) poff[L + 1] = poff[L] + c->h_plane_rows[L];
    const int nslot = c->nmap;                    // slots: the atom map (64-slot plane tiles)
    TRY(dalloc(c, &b.plane_off, poff.size()));
    HIP_TRY(c, hipMemcpy(b.plane_off, poff.data(), poff.size() * sizeof(int), hipMemcpyHostToDevice));
    {
      const int jchunks = std::max(1, std::min(64, (nslot + 1023) / 1024));
      int* cnt = nullptr;
      TRY(dalloc(c, &cnt, (size_t)jchunks * nslot));
      launch_ell_count(c->stream, nslot, jchunks, b.amap, b, p.Lx, p.Ly, c->Lz, p.rcut, cnt);
      TRY(launched(c, "ell count"));
      std::vector<int> h_cnt((size_t)jchunks * nslot);
      HIP_TRY(c, hipMemcpyAsync(h_cnt.data(), cnt, h_cnt.size() * sizeof(int), hipMemcpyDeviceToHost,
                                c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      int width = 0;
      for (int r = 0; r < nslot; ++r) {          // offsets: chunks of a row in order
        int o = 0;
        for (int ch = 0; ch < jchunks; ++ch) {
          const int k = h_cnt[(size_t)ch * nslot + r];
          h_cnt[(size_t)ch * nslot + r] = o;
          o += k;
        }
        width = std::max(width, o);
      }
      HIP_TRY(c, hipMemcpy(cnt, h_cnt.data(), h_cnt.size() * sizeof(int), hipMemcpyHostToDevice));
      width = (width + 7) / 8 * 8;                // the product reads 8 entries per step
      c->ell_width = width;
      dfree(c, b.ell_col);                        // a rebuild may change the width
      dfree(c, b.ell_val);
      TRY(dalloc(c, &b.ell_col, (size_t)width * nslot));
      TRY(dalloc(c, &b.ell_val, (size_t)width * nslot));
      launch_ell_fill(c->stream, nslot, jchunks, width, b.amap, cnt, b, p.Lx, p.Ly, c->Lz, p.rcut,
                      p.alpha, eta_ee, diag_self, b.ell_col, b.ell_val);
      TRY(launched(c, "ell fill"));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      dfree(c, cnt);
    }
    {
      // the ELL rows as dense 64 x 64 blocks of interacting slot tiles
      // (block columns ascending within a tile row)
      const int T = nslot / 64, width = c->ell_width;
      std::vector<int> hcol((size_t)width * nslot);
      std::vector<double> hval((size_t)width * nslot);
      HIP_TRY(c, hipMemcpy(hcol.data(), b.ell_col, hcol.size() * sizeof(int), hipMemcpyDeviceToHost));
      HIP_TRY(c, hipMemcpy(hval.data(), b.ell_val, hval.size() * sizeof(double), hipMemcpyDeviceToHost));
      std::vector<int> bptr(T + 1, 0), bcol, pos(T, -1);
      std::vector<double> bval;
      for (int I = 0; I < T; ++I) {
        std::vector<int> js;
        for (int r = I * 64; r < I * 64 + 64; ++r)
          for (int k = 0; k < width; ++k)
            if (hval[(size_t)r * width + k] != 0.0) {
              const int J = hcol[(size_t)r * width + k] / 64;
              if (pos[J] < 0) { pos[J] = 0; js.push_back(J); }
            }
        std::sort(js.begin(), js.end());
        const size_t base = bcol.size();
        for (size_t q = 0; q < js.size(); ++q) { pos[js[q]] = (int)(base + q); bcol.push_back(js[q]); }
        bval.resize(bcol.size() * 4096, 0.0);
        for (int r = I * 64; r < I * 64 + 64; ++r)
          for (int k = 0; k < width; ++k) {
            const double v = hval[(size_t)r * width + k];
            if (v == 0.0) continue;
            const int col = hcol[(size_t)r * width + k];
            bval[(size_t)pos[col / 64] * 4096 + (size_t)(r % 64) * 64 + col % 64] = v;
          }
        for (int J : js) pos[J] = -1;
        bptr[I + 1] = (int)bcol.size();
      }
      c->h_bdiag.assign(T, -1);
      for (int I = 0; I < T; ++I)
        for (int q = bptr[I]; q < bptr[I + 1]; ++q)
          if (bcol[q] == I) c->h_bdiag[I] = q;
      c->bsr_blocks = (int)bcol.size();
      dfree(c, b.bsr_col);
      dfree(c, b.bsr_val);
      TRY(dalloc(c, &b.bsr_col, bcol.size()));
      TRY(dalloc(c, &b.bsr_val, bval.size()));
      HIP_TRY(c, hipMemcpy(b.bsr_col, bcol.data(), bcol.size() * sizeof(int), hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(b.bsr_val, bval.data(), bval.size() * sizeof(double), hipMemcpyHostToDevice));
      dfree(c, b.ell_col);
      dfree(c, b.ell_val);
      // work items of the fused projection / real-space kernel: about 512
      // items of similar size (a unit: K = 64 of one 64 x 64 output tile)
      const int kunits = 2 * c->ncp / 64;
      const long U = (long)T * kunits + (long)bcol.size();
      const int u = (int)std::max<long>(4, (U + 511) / 512);
      std::vector<int> items;
      int nparts = 1;
      for (int I = 0; I < T; ++I) {
        int part = 0;
        const int nk = (kunits + u - 1) / u;
        for (int q = 0; q < nk; ++q)
          items.insert(items.end(), {I, 0, kunits * q / nk * 64, kunits * (q + 1) / nk * 64,
                                     part++, tplane[I]});
        const int nbI = bptr[I + 1] - bptr[I];
        const int nq = (nbI + u - 1) / u;
        for (int q = 0; q < nq; ++q)
          items.insert(items.end(), {I, 1, bptr[I] + nbI * q / nq, bptr[I] + nbI * (q + 1) / nq,
                                     part++, tplane[I]});
        nparts = std::max(nparts, part);
      }
      c->cg_nitems = (int)(items.size() / 6);
      c->cg_nparts = nparts;
      dfree(c, b.cg_items);
      TRY(dalloc(c, &b.cg_items, items.size()));
      HIP_TRY(c, hipMemcpy(b.cg_items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice));
      // plane sums split over each plane's slots to about 512 workgroups
      int q16 = 1 << 30;
      for (int L = 0; L < c->nlayers; ++L) q16 = std::min(q16, c->h_plane_rows[L] / 16);
      const int mt = 2 * c->ncp / 64;
      c->cg_ksplit = std::max(1, std::min({16, q16, (512 + mt * c->nlayers - 1) / (mt * c->nlayers)}));
    }
    TRY(dalloc(c, &b.dextra, (size_t)n));
    if (d_diag_extra)
      HIP_TRY(c, hipMemcpyAsync(b.dextra, d_diag_extra, (size_t)n * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream));
    else
      HIP_TRY(c, hipMemsetAsync(b.dextra, 0, (size_t)n * sizeof(double), c->stream));
    TRY(launched(c, "operator set-up"));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->op_background = background;
    c->have_op = true;
    return CPM_OK;
  }
  // A itself is assembled by its first consumer (cpm_invert on its stream,
  // so an asynchronous inversion also overlaps the assembly with b); only the
  // caller's diagonal term is copied now
  c->A_diag_extra = d_diag_extra != nullptr;
  if (d_diag_extra) {
    TRY(dalloc(c, &b.dextra, (size_t)n));
    HIP_TRY(c, hipMemcpyAsync(b.dextra, d_diag_extra, (size_t)n * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->A_pending = true;
  c->have_A = true;
  return CPM_OK;
}

}  // namespace

extern "C" {

cpm_status cpm_build_elastance(cpm_ctx* c, int n, const double* d_xyz, const int* d_eid, int n_e,
                               const double* d_diag_extra) {
  if (!c) return CPM_EINVAL;
  return build_impl(c, n, d_xyz, d_eid, n_e, d_diag_extra, true);
}

cpm_status cpm_build_operator(cpm_ctx* c, int n, const double* d_xyz, const int* d_eid, int n_e,
                              const double* d_diag_extra) {
  if (!c) return CPM_EINVAL;
  return build_impl(c, n, d_xyz, d_eid, n_e, d_diag_extra, false);
}

cpm_status cpm_invert(cpm_ctx* c, unsigned store_flags) {
  if (!c) return CPM_EINVAL;
  TRY(wait_invert(c));                    // a new inversion supersedes a pending one
  c->inv_failed = false;
  if (!c->have_A) return fail(c, CPM_ESTATE, "cpm_invert before cpm_build_elastance");
  if (store_flags & ~(unsigned)(CPM_STORE_F64 | CPM_STORE_F32 | CPM_STORE_BF16X2 | CPM_INVERT_ASYNC |
                                CPM_INVERT_FACTOR))
    return fail(c, CPM_EINVAL, "unknown store flags 0x%x", store_flags);
  const bool async = (store_flags & CPM_INVERT_ASYNC) != 0;
  const bool factor = (store_flags & CPM_INVERT_FACTOR) != 0;
  store_flags &= ~(unsigned)(CPM_INVERT_ASYNC | CPM_INVERT_FACTOR);
  if (factor && (store_flags & (CPM_STORE_F32 | CPM_STORE_BF16X2)))
    return fail(c, CPM_EINVAL, "CPM_INVERT_FACTOR keeps no copy of S");
  if (factor && c->n_e > CCM_MAXE)
    return fail(c, CPM_EUNSUPPORTED, "CPM_INVERT_FACTOR supports at most %d electrodes", CCM_MAXE);
  const int npad = c->npad, nb = npad / TILE;
  Buffers& b = c->b;
  TRY(dalloc(c, &b.L, (size_t)npad * npad));
  TRY(dalloc(c, &b.Dinv, (size_t)nb * TILE * TILE));
  TRY(ensure_inverse_buffers(c, store_flags, factor));
  c->factor_only = false;
  hipStream_t st = c->stream;
  if (async) {
    // a second stream of default priority, ordered after the work already
    // enqueued on the context stream (the assembly of A)
    if (!c->aux) {
      HIP_TRY(c, hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
      HIP_TRY(c, hipEventCreateWithFlags(&c->aux_ev, hipEventDisableTiming));
      HIP_TRY(c, hipEventCreateWithFlags(&c->main_ev, hipEventDisableTiming));
      HIP_TRY(c, hipHostMalloc((void**)&c->h_async, sizeof(*c->h_async), hipHostMallocDefault));
    }
    HIP_TRY(c, hipEventRecord(c->main_ev, c->stream));
    HIP_TRY(c, hipStreamWaitEvent(c->aux, c->main_ev, 0));
    st = c->aux;
  }
  TRY(assemble_A(c, st));
  HIP_TRY(c, hipMemcpyAsync(b.L, b.A, (size_t)npad * npad * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIP_TRY(c, hipMemsetAsync(b.flag, 0, sizeof(int), st));
  HIP_TRY(c, hipMemsetAsync(b.u, 0, npad * sizeof(double), st));
  // Blocked right-looking Cholesky on the lower triangle of L, two levels:
  // 64-wide panels inside blocks of OB columns (a multiple of 64), so that
  // the large trailing updates are rank-OB products (OB / 64 times fewer
  // passes over the trailing matrix than rank-64 ones).
  const int OB = c->chol_block;
  for (int K0 = 0; K0 < npad; K0 += OB) {
    const int kend = std::min(npad, K0 + OB);
    for (int k0 = K0; k0 < kend; k0 += TILE) {
      const int kb = k0 / TILE, rest = npad - k0 - TILE;
      double* diag = b.L + (size_t)k0 * npad + k0;
      { Timed t(c, "potrf_diag", st);
        launch_potrf_diag(st, diag, npad, b.Dinv + (size_t)kb * TILE * TILE, b.flag, k0); }
      if (rest > 0) {
        Timed t(c, "chol_update", st);
        double* panel = b.L + (size_t)(k0 + TILE) * npad + k0;
        // L21 = A21 L11^-T for every row below the panel
        launch_gemm_f64(st, false, true, rest, TILE, TILE, 1.0, panel, npad,
                        b.Dinv + (size_t)kb * TILE * TILE, TILE, 0.0, panel, npad, 0, 0);
        // A22 -= L21 L21^T on the block's own remaining columns (lower tiles)
        const int pw = kend - (k0 + TILE);
        if (pw > 0) {
          double* trail = b.L + (size_t)(k0 + TILE) * npad + (k0 + TILE);
          launch_gemm_f64(st, false, true, rest, pw, TILE, -1.0, panel, npad, panel, npad, 1.0,
                          trail, npad, 1, 0);
        }
      }
      TRY(launched(c, "cholesky"));
    }
    // the columns right of the block: A22 -= L21 L21^T with the block's OB columns
    const int rest = npad - kend;
    if (rest > 0) {
      Timed t(c, "chol_update", st);
      const double* P = b.L + (size_t)kend * npad + K0;
      launch_gemm_f64(st, false, true, rest, rest, kend - K0, -1.0, P, npad, P, npad, 1.0,
                      b.L + (size_t)kend * npad + kend, npad, 1, 0);
      TRY(launched(c, "cholesky"));
    }
  }
  if (!async) {
    int flag = 0;
    HIP_TRY(c, hipMemcpyAsync(&flag, b.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (flag != 0) {
      c->pivot = flag - 1;
      c->have_inv = false;
      return fail(c, CPM_ENOTPD, "elastance matrix not positive definite at pivot %d", c->pivot);
    }
  }
  if (factor) {
    // keep L: u, s and S G from triangular solves, no L^-1 or A^-1
    TRY(factor_response(c, st));
    c->store = CPM_STORE_F64;
  } else {
    // X = L^-1 by blocked forward substitution (X stored in Ainv's buffer
    // first), grouped like the factorisation: row blocks of 64 inside blocks
    // of OB rows, the rows below a block updated by one rank-OB product
    double* X = b.Ainv;
    launch_set_identity(st, npad, X);
    for (int K0 = 0; K0 < npad; K0 += OB) {
      const int kend = std::min(npad, K0 + OB);
      for (int k0 = K0; k0 < kend; k0 += TILE) {
        const int kb = k0 / TILE, cols = k0 + TILE, rin = kend - k0 - TILE;
        double* Xk = X + (size_t)k0 * npad;
        Timed t(c, "trtri", st);
        // X_k = L_kk^-1 X_k on the columns that can be non-zero
        launch_gemm_f64(st, false, false, TILE, cols, TILE, 1.0, b.Dinv + (size_t)kb * TILE * TILE,
                        TILE, Xk, npad, 0.0, Xk, npad, 0, 0);
        if (rin > 0) {
          // the block's rows below: X_i -= L_ik X_k
          launch_gemm_f64(st, false, false, rin, cols, TILE, -1.0,
                          b.L + (size_t)(k0 + TILE) * npad + k0, npad, Xk, npad, 1.0,
                          X + (size_t)(k0 + TILE) * npad, npad, 0, 0);
        }
        TRY(launched(c, "trtri"));
      }
      const int rest = npad - kend;
      if (rest > 0) {
        // every row below the block: X_below -= L_below,block X_block (columns < kend)
        Timed t(c, "trtri", st);
        launch_gemm_f64(st, false, false, rest, kend, kend - K0, -1.0,
                        b.L + (size_t)kend * npad + K0, npad, X + (size_t)K0 * npad, npad, 1.0,
                        X + (size_t)kend * npad, npad, 0, 0);
        TRY(launched(c, "trtri"));
      }
    }
    // A^-1 = X^T X (lower tiles, k from max(row, col)), result into L's buffer,
    // then swap names so Ainv holds A^-1
    { Timed t(c, "lauum", st);
      launch_gemm_f64(st, true, false, npad, npad, npad, 1.0, X, npad, X, npad, 0.0, b.L, npad, 1, 1);
      launch_mirror_lower(st, npad, b.L); }
    TRY(launched(c, "lauum"));
    std::swap(b.L, b.Ainv);
    TRY(form_S(c, st, store_flags));
  }
  c->factor_only = factor;
  if (async) {
    // results are joined by the first call that needs them (finish_invert)
    HIP_TRY(c, hipMemcpyAsync(&c->h_async->s, b.scal, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipMemcpyAsync(&c->h_async->flag, b.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipEventRecord(c->aux_ev, st));
    c->inv_pending = true;
    c->have_inv = true;
    return CPM_OK;
  }
  HIP_TRY(c, hipMemcpyAsync(&c->s_sum, b.scal, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(c, hipStreamSynchronize(st));
  c->have_inv = true;
  return CPM_OK;
}

cpm_status cpm_set_potential(cpm_ctx* c, const double* h_v_electrode) {
  if (!c) return CPM_EINVAL;
  TRY(finish_invert(c));
  if (!c->have_inv && !c->have_op) return fail(c, CPM_ESTATE, "cpm_set_potential before cpm_invert");
  if (!h_v_electrode) return fail(c, CPM_EINVAL, "h_v_electrode is NULL");
  for (int a = 0; a < c->n_e; ++a)
    if (!std::isfinite(h_v_electrode[a])) return fail(c, CPM_EINVAL, "potential %d not finite", a);
  c->h_v.assign(h_v_electrode, h_v_electrode + c->n_e);
  TRY(ensure_vat(c));
  if (c->n_e <= CCM_MAXE && (c->b.sg || !c->have_inv)) {
    // v = G v~ and d = (S G) v~ from the cached response (Eq. 6): one small
    // kernel, the potentials passed by value, nothing copied or awaited
    ElectrodeValues vt{};
    for (int a = 0; a < c->n_e; ++a) vt.v[a] = c->h_v[a];
    launch_apply_potential(c->stream, c->n, c->npad, c->n_e, c->b.eid,
                           c->have_inv ? c->b.sg : nullptr, vt, c->b.vat, c->b.d);
    TRY(launched(c, "set_potential"));
    c->have_v = true;
    return CPM_OK;
  }
  std::vector<double> vat(c->npad, 0.0);
  for (int i = 0; i < c->n; ++i) vat[i] = c->h_v[c->h_eid[i]];
  HIP_TRY(c, hipMemcpyAsync(c->b.vat, vat.data(), c->npad * sizeof(double), hipMemcpyHostToDevice, c->stream));
  // d = S v (more electrodes than the cached response holds)
  if (c->have_inv)
    launch_matvec(c->stream, 0, c->npad, c->b.S, 1, c->b.vat, nullptr, 0, 0.0, c->b.d, c->npad, 0);
  TRY(launched(c, "set_potential"));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->have_v = true;
  return CPM_OK;
}

cpm_status cpm_set_field(cpm_ctx* c, double dv0, int bottom) {
  if (!c) return CPM_EINVAL;
  TRY(finish_invert(c));
  if (!c->have_inv && !c->have_op) return fail(c, CPM_ESTATE, "cpm_set_field before cpm_invert");
  if (c->p.geometry != CPM_GEOM_3D)
    return fail(c, CPM_EUNSUPPORTED, "the finite-field method needs the 3D-periodic cell (geometry 2)");
  if (!std::isfinite(dv0)) return fail(c, CPM_EINVAL, "dv0 not finite");
  if (bottom < 0 || bottom >= c->n_e)
    return fail(c, CPM_EINVAL, "bottom electrode %d outside [0, %d)", bottom, c->n_e);
  Buffers& b = c->b;
  TRY(ensure_vat(c));
  if (!b.zeta || c->field_bottom != bottom) {
    // zeta_i = z_i / Lz, plus one cell for the bottom electrode (Sec. II.F:
    // normalised z positions with the bottom electrode offset, so that the
    // two electrodes meet across the periodic z boundary as one conductor)
    TRY(dalloc(c, &b.zeta, (size_t)c->npad));
    std::vector<double> z(c->npad, 0.0);
    for (int i = 0; i < c->n; ++i)
      z[i] = c->h_xyz[3 * i + 2] / c->Lz + (c->h_eid[i] == bottom ? 1.0 : 0.0);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(b.zeta, z.data(), z.size() * sizeof(double), hipMemcpyHostToDevice));
    c->field_bottom = bottom;
    c->szeta_ok = false;
  }
  if (c->have_inv && !c->szeta_ok) {
    // S zeta once per inverse (Eq. 14 with the response cached): a new dv0
    // then costs O(n)
    TRY(dalloc(c, &b.szeta, (size_t)c->npad));
    TRY(apply_S_one(c, b.zeta, b.szeta));
    c->szeta_ok = true;
  }
  launch_scale_field(c->stream, c->npad, dv0, b.zeta, c->have_inv ? b.szeta : nullptr, b.vat, b.d);
  TRY(launched(c, "set_field"));
  c->h_v.clear();
  c->have_v = true;
  return CPM_OK;
}

cpm_status cpm_set_potential_atoms(cpm_ctx* c, const double* h_v) {
  if (!c) return CPM_EINVAL;
  TRY(finish_invert(c));
  if (!c->have_inv && !c->have_op)
    return fail(c, CPM_ESTATE, "cpm_set_potential_atoms before cpm_invert");
  if (!h_v) return fail(c, CPM_EINVAL, "h_v is NULL");
  for (int i = 0; i < c->n; ++i)
    if (!std::isfinite(h_v[i])) return fail(c, CPM_EINVAL, "potential of atom %d not finite", i);
  c->h_v.clear();
  std::vector<double> vat(c->npad, 0.0);
  for (int i = 0; i < c->n; ++i) vat[i] = h_v[i];
  TRY(ensure_vat(c));
  HIP_TRY(c, hipMemcpyAsync(c->b.vat, vat.data(), c->npad * sizeof(double), hipMemcpyHostToDevice, c->stream));
  if (c->have_inv) TRY(apply_S_one(c, c->b.vat, c->b.d));
  TRY(launched(c, "set_potential_atoms"));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->have_v = true;
  return CPM_OK;
}

}  // extern "C"

namespace {

// validation and (first-use) allocation for cpm_potential_vector
// the real-space stream and its two events, created on first use (default
// priority, like every stream of the library)
cpm_status ensure_rs_stream(cpm_ctx* c) {
  if (c->rs_stream) return CPM_OK;
  HIP_TRY(c, hipStreamCreateWithFlags(&c->rs_stream, hipStreamNonBlocking));
  HIP_TRY(c, hipEventCreateWithFlags(&c->rs_ev_in, hipEventDisableTiming));
  HIP_TRY(c, hipEventCreateWithFlags(&c->rs_ev_out, hipEventDisableTiming));
  return CPM_OK;
}

cpm_status pv_prepare(cpm_ctx* c, int batch, const double* d_xyz, void* d_b, int b_is_f32) {
  if (!(c->have_A || c->have_op) || !c->have_elyt)
    return fail(c, CPM_ESTATE, "cpm_potential_vector needs cpm_set_electrolyte and cpm_build_elastance");
  if (batch <= 0 || !d_b || (c->m > 0 && !d_xyz))
    return fail(c, CPM_EINVAL, "need batch > 0 and non-NULL buffers");
  if (b_is_f32 != 0 && b_is_f32 != 1) return fail(c, CPM_EINVAL, "b_is_f32 must be 0 or 1");
  TRY(ensure_uploaded(c));
  TRY(ensure_step_buffers(c));
  if (c->rs_conc_ok) TRY(ensure_rs_stream(c));
  return CPM_OK;
}

// kernel launches of cpm_potential_vector (no allocation, copy or memset)
cpm_status pv_enqueue(cpm_ctx* c, int batch, const double* d_xyz, void* d_b, int b_is_f32) {
  const cpm_params& p = c->p;
  const int n = c->n, m = c->m;
  const size_t esz = b_is_f32 ? sizeof(float) : sizeof(double);
  Buffers& b = c->b;
  hipStream_t st = c->stream;
  // FP64 structure factors on matrix cores unless switched off; planar
  // electrodes then take the grouped path (pv_group configurations per
  // launch, k_z folded into the planes, projection fused into the combine)
  const bool mfma = c->sf_mfma && c->use_sf_mfma;
  const bool fast = mfma && c->nlayers > 0 && batch >= c->pv_fast_min;
  // b stored in FP32 (the reduced-precision solve path): structure factors on
  // FP32 matrix cores, FP32 phase tables (switch: CPM_SF_FP32=0)
  const int sf32 = (b_is_f32 && c->sf32_ok) ? (c->sf16_ok ? 2 : 1) : 0;
  const int G = fast ? c->pv_group : 1;
  const int mpad64 = std::max(64, (m + 63) / 64 * 64);
  // the charges ordered by z (from the first configuration of a large
  // batch) for the real-space pass, so that whole blocks fall outside the
  // planes' windows; small batches (a single configuration per MD step)
  // reuse the last order: the block z ranges come from the actual positions,
  // so an order that has aged only costs skipped blocks, never a pair
  const int* perm = nullptr;
  if (m > 0 && (batch >= c->rs_sort_min || !c->zperm_ok)) {
    Timed t(c, "zsort");
    launch_zsort(st, m, d_xyz, c->Lz, zsort_bins(c->Lz), b.zperm);
    c->zperm_ok = true;
  }
  if (m > 0 && c->zperm_ok) perm = b.zperm;
  for (int s0 = 0; s0 < batch; s0 += G) {
    const int g = std::min(G, batch - s0);
    const double* xyz = d_xyz ? d_xyz + (size_t)s0 * m * 3 : nullptr;
    void* out = static_cast<char*>(d_b) + (size_t)s0 * n * esz;
    if (m == 0) {
      launch_fill_zero(st, (size_t)g * n * esz / sizeof(float), static_cast<float*>(out));
      continue;
    }
    const int nch = mfma ? sf_chunks_for(c, g, sf32 == 2) : 0;
    const int rch = fast ? rchunks_for(c, g) : c->rchunks;
    // grouped path: the real-space pass runs on its own stream beside the
    // structure factors (VALU/LDS-bound beside MFMA-bound work); it starts
    // after everything enqueued so far (the previous group's final sum,
    // which read its partials) and the final sum of this group waits for it
    const bool conc = fast && c->rs_stream && !c->capturing;
    hipStream_t rst = st;
    if (conc) {
      HIP_TRY(c, hipEventRecord(c->rs_ev_in, st));
      HIP_TRY(c, hipStreamWaitEvent(c->rs_stream, c->rs_ev_in, 0));
      rst = c->rs_stream;
    }
    { Timed t(c, "real_space_b", rst);
      launch_gather_charges(rst, g, m, mpad64, perm, xyz, b.elq, p.Lx, p.Ly, b.cq, b.zr);
      launch_b_real_space(rst, g, n, m, mpad64, rch, b, c->nmap, b.cq, b.zr, p.Lx, p.Ly, c->Lz,
                          p.rcut, b.phir_part, fast ? rs_target(c) : 512,
                          rs_plane(c) ? b.ptab : nullptr); }
    if (conc) HIP_TRY(c, hipEventRecord(c->rs_ev_out, rst));
    if (!mfma) {
      Timed t(c, "dipole");
      launch_b_elyt_dipole(st, g, m, xyz, b.elq, b.dip);
    }
    if (mfma) {
      // the table kernel also writes the dipole partials
      { Timed t(c, "sf_tables");
        launch_b_sf_tables(st, g, m, c->mpad, c->nxm, c->nym, c->sfm_nbz, xyz, b.elq, p.Lx, p.Ly,
                           c->Lz, b.sft, sf32, b.dip); }
      { Timed t(c, "structure_factor");
        launch_b_sf_mfma(st, g, c->mpad, nch, sf32 == 2 ? c->sf16_nitems : c->sfm_nitems,
                         sf32 == 2 ? b.sf16_items : b.sfm_items, b.sc_nx, b.sc_ny,
                         c->ncolsort, c->nxm, c->nym, c->sfm_nbz, b.sft, b.tile_nb, b.tile_off,
                         c->sfm_pchunk, b.sfm_part, sf32, c->sf16_nt); }
    } else {
      { Timed t(c, "structure_factor");
        launch_b_structure_factor(st, b_is_f32, c->nruns, b.runs, c->nk, m, c->mchunks, xyz,
                                  b.elq, p.Lx, p.Ly, c->Lz, c->nxm, c->nym, c->nzm, b.sf_part); }
      { Timed t(c, "sf_reduce");
        launch_b_sf_reduce(st, c->nk, c->mchunks, b.sf_part, b.w2, b.sfw); }
    }
    if (fast) {
      { Timed t(c, "sf_reduce");
        launch_b_sf_layer_reduce(st, g, c->ncolsort, nch, c->sfm_pchunk, c->nlayers,
                                 c->sfm_npadc / 2, c->sfm_maxcnt, b.tile_nb, b.tile_off, b.sc_lo,
                                 b.sc_len, b.sc_koff, b.sc_nidx, b.sfm_part, b.w2, b.pz,
                                 2 * c->ncp, b.bT); }
      { Timed t(c, "projection");
        // one configuration: vector units (a matrix-core tile would fill 64 lanes for one)
        if (g == 1)
          launch_proj_one(st, c->b_nitems, c->nmap, c->ncp, b.b_items, b.Ecat, b.bT, b.bPhi);
        else
          launch_cg_tiles(st, c->b_nitems, c->nmap, c->ncp, b.b_items, b.Ecat, b.bT, nullptr,
                          nullptr, nullptr, b.bPhi); }
      if (conc) HIP_TRY(c, hipStreamWaitEvent(st, c->rs_ev_out, 0));
      { Timed t(c, "combine");
        launch_b_final(st, g, n, c->nmap, c->b_nparts, b.slot_of, b.bPhi, b.phir_part,
                       rch, b, b.dip, c->dip_blocks, c->cdip, c->ke, out, b_is_f32); }
      TRY(launched(c, "potential_vector"));
      continue;
    }
    // general path, one configuration (g == 1)
    if (mfma) {
      Timed t(c, "sf_reduce");
      launch_b_sf_mfma_reduce(st, c->ncolsort, nch, c->sfm_pchunk, b.tile_nb, b.tile_off, b.sc_lo,
                              b.sc_len, b.sc_koff, b.sc_nidx, c->sfm_ntot, b.sfm_part, b.w2,
                              b.sfw);
    }
    int kparts = c->kchunks;
    if (c->nlayers > 0) {
      Timed t(c, "kspace_project");
      launch_b_layer_project(st, n, (int)c->h_cols.size(), c->nlayers, b.cols, b.layer_of,
                             b.layer_fz, b, b.sfw, b.layerT, b.phik_part);
      kparts = layer_project_chunks((int)c->h_cols.size());
    } else {
      Timed t(c, "kspace_project");
      launch_b_kspace_project(st, b_is_f32, n, c->kchunks, b.cols, b.chunk_col, b, b.sfw,
                              b.phik_part);
    }
    { Timed t(c, "combine");
      launch_b_combine(st, n, kparts, c->rchunks, b.phik_part, b.phir_part, b, b.dip,
                       c->dip_blocks, c->cdip, c->ke, out, b_is_f32); }
    TRY(launched(c, "potential_vector"));
  }
  return CPM_OK;
}

// validation of cpm_solve_charges' arguments and state (no allocation)
cpm_status sc_validate(cpm_ctx* c, int batch, const void* d_b, int b_is_f32, unsigned mode,
                       double* d_q) {
  TRY(finish_invert(c));
  if (!c->have_inv) return fail(c, CPM_ESTATE, "cpm_solve_charges before cpm_invert");
  if (!c->have_v) return fail(c, CPM_ESTATE, "cpm_solve_charges before cpm_set_potential");
  if (batch <= 0 || !d_b || !d_q) return fail(c, CPM_EINVAL, "need batch > 0 and non-NULL b, q");
  if (b_is_f32 != 0 && b_is_f32 != 1) return fail(c, CPM_EINVAL, "b_is_f32 must be 0 or 1");
  const unsigned prec = mode & 0xffu;
  if ((mode & ~0x3ffu) != 0 || prec > 2) return fail(c, CPM_EINVAL, "unknown solve mode 0x%x", mode);
  if (mode & CPM_SOLVE_CCM) {
    if (prec != 0 || (mode & CPM_SOLVE_REFINE))
      return fail(c, CPM_EUNSUPPORTED, "constrained charges run in FP64 without refinement");
    if (!c->have_q) return fail(c, CPM_ESTATE, "CPM_SOLVE_CCM before cpm_set_charge");
  }
  if (c->factor_only && mode != CPM_SOLVE_F64)
    return fail(c, CPM_ESTATE, "the factor-only inverse (CPM_INVERT_FACTOR) solves in mode 0 only");
  if (prec == 1 && !(c->store & CPM_STORE_F32)) return fail(c, CPM_EINVAL, "FP32 copy of S not kept");
  if (prec == 2 && !(c->store & CPM_STORE_BF16X2))
    return fail(c, CPM_EINVAL, "split-BF16 copy of S not kept");
  return CPM_OK;
}

// validation and (first-use) allocation for cpm_solve_charges
cpm_status sc_prepare(cpm_ctx* c, int batch, const void* d_b, int b_is_f32, unsigned mode,
                      double* d_q) {
  TRY(sc_validate(c, batch, d_b, b_is_f32, mode, d_q));
  const unsigned prec = mode & 0xffu;
  const bool gemm = (batch >= GEMM_MIN_BATCH && prec == 0) || prec == 2 || c->factor_only;
  const int rows = gemm ? ((batch + TILE - 1) / TILE) * TILE : batch;
  TRY(ensure_solve_buffers(c, rows));
  if (prec == 2) {
    const cpm_ctx::GemmCfg cfg = bf16_cfg(c, rows);
    if (cfg.ks > 1) TRY(ensure_kpart(c, (size_t)cfg.ks * rows * c->npad));
  }
  return CPM_OK;
}

// kernel launches of cpm_solve_charges (no allocation, copy or memset)
cpm_status sc_enqueue(cpm_ctx* c, int batch, const void* d_b, int b_is_f32, unsigned mode,
                      double* d_q, double* d_Qe, const SolveWork& w) {
  if (batch <= 0 || !d_b || !d_q) return fail(c, CPM_EINVAL, "need batch > 0 and non-NULL b, q");
  if (b_is_f32 != 0 && b_is_f32 != 1) return fail(c, CPM_EINVAL, "b_is_f32 must be 0 or 1");
  const unsigned prec = mode & 0xffu;
  const bool refine = (mode & CPM_SOLVE_REFINE) != 0;
  const int n = c->n, npad = c->npad;
  // split-BF16 always runs on matrix cores (rows padded to 64); FP64 from
  // GEMM_MIN_BATCH vectors on; FP32 streams S32 per vector
  const bool gemm = (batch >= GEMM_MIN_BATCH && prec == 0) || prec == 2;
  const int rows = gemm ? ((batch + TILE - 1) / TILE) * TILE : batch;
  Buffers& b = c->b;
  hipStream_t st = c->stream;
  const void* Sm = (prec == 1) ? (const void*)b.S32 : (const void*)b.S;
  const int which = (prec == 1) ? 1 : 0;
  const char* mv_name = (prec == 1) ? "matvec_f32" : "matvec_f64";

  if (c->factor_only) {
    // S (b + v) = P A^-1 b + d: the batch as rows (padded to 64), A^-1 by
    // substitution with the Cholesky factor, then P and d in the finalize
    const int frows = ((batch + TILE - 1) / TILE) * TILE;
    { Timed t(c, "pad_rows");
      launch_pad_rows(st, n, npad, batch, frows, d_b, b_is_f32, nullptr, w.bpad); }
    TRY(factor_solve_rows(c, st, frows, w.bpad, w.qpad));
    { Timed t(c, "finalize");
      launch_finalize(st, n, batch, w.bpad, npad, b.d, b.u, b.scal, b.eid, c->n_e, d_q, n, d_Qe); }
    return launched(c, "solve (factor)");
  }

  if (mode & CPM_SOLVE_CCM) {
    // constrained charges (Eq. 7): y = A^-1 b in FP64, then the per-electrode
    // correction q = y + U C~^-1 (Q - G^T y)
    if (!gemm) {
      { Timed t(c, "pad_rows");
        launch_center_pad(st, n, npad, batch, d_b, b_is_f32, n, 0, w.bpad); }
      Timed t(c, "matvec_f64");
      launch_matvec(st, 0, npad, b.Ainv, batch, w.bpad, nullptr, 0, 0.0, w.qt, npad, 0);
    } else {
      { Timed t(c, "pad_rows");
        launch_pad_rows(st, n, npad, batch, rows, d_b, b_is_f32, nullptr, w.bpad); }
      Timed t(c, "gemm_f64");
      launch_gemm_f64(st, false, false, rows, npad, npad, 1.0, w.bpad, npad, b.Ainv, npad, 0.0, w.qt,
                      npad, 0, 0);
    }
    { Timed t(c, "finalize");
      launch_ccm_finalize(st, n, batch, w.qt, npad, b.ccmU, b.ccmC, b.ccmC + c->n_e * c->n_e, b.eid,
                          c->n_e, d_q, n, d_Qe); }
    return launched(c, "solve (constrained charges)");
  }

  // S~ x for a batch stored row-wise (stride npad) -> y (stride npad) (+ add)
  auto apply_S = [&](const double* x, double* y, bool accumulate) {
    if (prec == 0) {
      Timed t(c, "gemm_f64");
      launch_gemm_f64(st, false, false, rows, npad, npad, 1.0, x, npad, b.S, npad,
                      accumulate ? 1.0 : 0.0, y, npad, 0, 0);
    } else {
      Timed t(c, "gemm_bf16x3");
      enqueue_bf16(c, x, y, rows, accumulate, w.bf16 ? *w.bf16 : bf16_cfg(c, rows), w);
    }
  };

  // Every product with S~ acts on a centred vector: S e = 0 makes that exact,
  // and it keeps the rounding of a low-precision S~ away from the large
  // uniform part of b and of the refinement residual.
  if (!gemm) {
    // q~ = S~ (b - mean(b) e) + d, one streaming pass over S~ per vector
    { Timed t(c, "row_means");
      launch_center_pad(st, n, npad, batch, d_b, b_is_f32, n, 1, w.bpad); }
    { Timed t(c, mv_name);
      launch_matvec(st, which, npad, Sm, batch, w.bpad, b.d, 0, 1.0, w.qt, npad, 0); }
    if (!refine) {
      Timed t(c, "finalize");
      launch_finalize(st, n, batch, w.qt, npad, nullptr, b.u, b.scal, b.eid, c->n_e, d_q, n, d_Qe);
      return launched(c, "solve");
    }
    // one refinement step (FP64 except the products with S~):
    //   qp = P q~ (P: neutrality projection), r = (b + v) - A qp, q = P (qp + S~ r).
    // Valid because S A qp = qp when e^T qp = 0.
    { Timed t(c, "finalize");
      launch_finalize(st, n, batch, w.qt, npad, nullptr, b.u, b.scal, b.eid, c->n_e, w.qpad, npad,
                      nullptr); }
    { Timed t(c, "make_rhs");
      launch_make_rhs(st, n, npad, batch, d_b, b_is_f32, b.vat, w.res); }
    { Timed t(c, "matvec_f64");
      launch_matvec(st, 0, npad, b.A, batch, w.qpad, w.res, npad, 1.0, w.qt, npad, 1); }
    { Timed t(c, "center_rows");
      launch_center_rows(st, n, npad, batch, w.qt); }
    { Timed t(c, mv_name);
      launch_matvec(st, which, npad, Sm, batch, w.qt, w.qpad, npad, 1.0, w.res, npad, 0); }
    { Timed t(c, "finalize");
      launch_finalize(st, n, batch, w.res, npad, nullptr, b.u, b.scal, b.eid, c->n_e, d_q, n, d_Qe); }
    return launched(c, "solve (refined)");
  }

  // batched: Q~ = B S~ as one MFMA GEMM over all vectors (rows padded to 64)
  { Timed t(c, "row_means");
    launch_row_means(st, n, batch, d_b, b_is_f32, n, w.means); }
  { Timed t(c, "pad_rows");
    launch_pad_rows(st, n, npad, batch, rows, d_b, b_is_f32, w.means, w.bpad); }
  apply_S(w.bpad, w.qpad, false);
  if (!refine) {
    Timed t(c, "finalize");
    launch_finalize(st, n, batch, w.qpad, npad, b.d, b.u, b.scal, b.eid, c->n_e, d_q, n, d_Qe);
    return launched(c, "solve (batched)");
  }
  { Timed t(c, "finalize");
    launch_finalize(st, n, batch, w.qpad, npad, b.d, b.u, b.scal, b.eid, c->n_e, w.qt, npad,
                    nullptr); }
  { Timed t(c, "make_rhs");
    launch_make_rhs(st, n, npad, batch, d_b, b_is_f32, b.vat, w.res); }
  // R = C - Qp A (FP64 MFMA), centred, then Q = Qp + R S~
  { Timed t(c, "gemm_f64");
    launch_gemm_f64(st, false, false, rows, npad, npad, -1.0, w.qt, npad, b.A, npad, 1.0, w.res,
                    npad, 0, 0); }
  { Timed t(c, "center_rows");
    launch_center_rows(st, n, npad, batch, w.res); }
  apply_S(w.res, w.qt, true);
  { Timed t(c, "finalize");
    launch_finalize(st, n, batch, w.qt, npad, nullptr, b.u, b.scal, b.eid, c->n_e, d_q, n, d_Qe); }
  return launched(c, "solve (batched, refined)");
}

}  // namespace

extern "C" {

cpm_status cpm_potential_vector(cpm_ctx* c, int batch, const double* d_xyz, void* d_b, int b_is_f32) {
  if (!c) return CPM_EINVAL;
  TRY(pv_prepare(c, batch, d_xyz, d_b, b_is_f32));
  return pv_enqueue(c, batch, d_xyz, d_b, b_is_f32);
}

cpm_status cpm_solve_charges(cpm_ctx* c, int batch, const void* d_b, int b_is_f32, unsigned mode,
                             double* d_q, double* d_Qe) {
  if (!c) return CPM_EINVAL;
  TRY(sc_prepare(c, batch, d_b, b_is_f32, mode, d_q));
  return sc_enqueue(c, batch, d_b, b_is_f32, mode, d_q, d_Qe, ctx_work(c));
}

}  // extern "C"

// the fixed work array of cpm_solve_charges_noalloc (one per GPU)
static __device__ __align__(256) double scratch[CPM_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

// ---- solve without allocation (cpm_solve_charges_noalloc) -----------------
// The work buffers live in one fixed device array per GPU.  Host code never
// uses the array's name as an address: its device address is looked up once
// per device with hipGetSymbolAddress (with that device current) and kept.
constexpr size_t NOALLOC_BYTES = (size_t)CPM_NOALLOC_SCRATCH_BYTES;

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_dev[NOALLOC_MAX_DEVICES] = {};

cpm_status scratch_address(cpm_ctx* c, double** out) {
  int dev = -1;
  HIP_TRY(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(c, CPM_EUNSUPPORTED, "device %d beyond the %d the scratch table holds", dev,
                NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, CPM_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = scratch_dev[dev];
  return CPM_OK;
}

}  // namespace

extern "C" {

cpm_status cpm_solve_charges_noalloc(cpm_ctx* c, int batch, const void* d_b, int b_is_f32,
                                     unsigned mode, double* d_q, double* d_Qe) {
  if (!c) return CPM_EINVAL;
  TRY(sc_validate(c, batch, d_b, b_is_f32, mode, d_q));
  if (c->factor_only) return fail(c, CPM_ESTATE, "the no-allocation solve needs S (not CPM_INVERT_FACTOR)");
  const unsigned prec = mode & 0xffu;
  const bool gemm = (batch >= GEMM_MIN_BATCH && prec == 0) || prec == 2;
  const size_t rows = gemm ? ((size_t)(batch + TILE - 1) / TILE) * TILE : (size_t)batch;
  const size_t sz = rows * c->npad;              // doubles per work matrix
  // qt, res, qpad, bpad (FP64), the BF16 pairs of the left operand (half a
  // matrix of doubles each), the row means (rounded to 256 bytes)
  const size_t means = (rows + 31) / 32 * 32;
  const size_t need = 4 * sz + (gemm ? sz : 0) + means;
  if (need * sizeof(double) > NOALLOC_BYTES)
    return fail(c, CPM_EINVAL,
                "batch %d at n = %d needs %zu bytes of work space, more than the %zu of the fixed "
                "scratch array; use cpm_solve_charges", batch, c->n, need * sizeof(double),
                NOALLOC_BYTES);
  double* base = nullptr;
  TRY(scratch_address(c, &base));
  SolveWork w{};
  w.qt = base;
  w.res = base + sz;
  w.qpad = base + 2 * sz;
  w.bpad = base + 3 * sz;
  w.means = base + 4 * sz;
  w.xhi = gemm ? reinterpret_cast<uint16_t*>(base + 4 * sz + means) : nullptr;
  w.xlo = gemm ? w.xhi + sz : nullptr;
  w.kpart = nullptr;
  cpm_ctx::GemmCfg cfg = bf16_cfg(c, (int)rows);
  if (cfg.ks != 1) { cfg.ks = 1; cfg.grid = 0; }   // no split-K partials
  w.bf16 = &cfg;
  // the array keeps the previous call's contents: clear it (a fill kernel,
  // so the call can also sit inside a captured graph)
  launch_fill_zero(c->stream, need * 2, reinterpret_cast<float*>(base));
  TRY(launched(c, "scratch clear"));
  const bool timing = c->timing;
  c->timing = false;                              // no event creation on this path
  const cpm_status st = sc_enqueue(c, batch, d_b, b_is_f32, mode, d_q, d_Qe, w);
  c->timing = timing;
  return st;
}

cpm_status cpm_capture_step(cpm_ctx* c, int batch, const double* d_xyz, void* d_b, int b_is_f32,
                            unsigned mode, double* d_q, double* d_Qe) {
  if (!c) return CPM_EINVAL;
  if (!c->stream)
    return fail(c, CPM_EINVAL, "graph capture needs a non-default stream for the context");
  TRY(pv_prepare(c, batch, d_xyz, d_b, b_is_f32));
  TRY(sc_prepare(c, batch, d_b, b_is_f32, mode, d_q));
  if (c->factor_only) return fail(c, CPM_ESTATE, "graph capture needs S (not CPM_INVERT_FACTOR)");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
  if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
  const bool timing = c->timing;
  c->timing = false;                               // no event nodes in the graph
  HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  c->capturing = true;                             // one stream in the graph
  cpm_status st = pv_enqueue(c, batch, d_xyz, d_b, b_is_f32);
  c->capturing = false;
  if (st == CPM_OK) st = sc_enqueue(c, batch, d_b, b_is_f32, mode, d_q, d_Qe, ctx_work(c));
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &g);
  c->timing = timing;
  if (st != CPM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(c, CPM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  c->graph = g;
  HIP_TRY(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
  c->graph_gen = c->alloc_gen;
  const unsigned prec = mode & 0xffu;
  c->graph_store = prec == 1 ? CPM_STORE_F32 : prec == 2 ? CPM_STORE_BF16X2 : CPM_STORE_F64;
  c->graph_ccm = (mode & CPM_SOLVE_CCM) != 0;
  return CPM_OK;
}

cpm_status cpm_replay_step(cpm_ctx* c) {
  if (!c) return CPM_EINVAL;
  TRY(finish_invert(c));
  if (!c->graph_exec) return fail(c, CPM_ESTATE, "cpm_replay_step before cpm_capture_step");
  // the graph holds raw device addresses: any reallocation since capture
  // (a larger eager batch, a rebuild) or a dropped copy of S invalidates it
  if (c->alloc_gen != c->graph_gen || !c->have_inv || !c->have_v ||
      (c->store & c->graph_store) != c->graph_store || (c->graph_ccm && !c->have_q))
    return fail(c, CPM_ESTATE, "context buffers changed since cpm_capture_step; capture again");
  HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
  return CPM_OK;
}

cpm_status cpm_set_charge(cpm_ctx* c, const double* h_Q) {
  if (!c) return CPM_EINVAL;
  TRY(finish_invert(c));
  if (!c->have_inv) return fail(c, CPM_ESTATE, "cpm_set_charge before cpm_invert");
  if (c->factor_only) return fail(c, CPM_ESTATE, "constrained charges need A^-1 (not CPM_INVERT_FACTOR)");
  if (!h_Q) return fail(c, CPM_EINVAL, "h_Q is NULL");
  const int ne = c->n_e, n = c->n;
  if (ne > CCM_MAXE) return fail(c, CPM_EUNSUPPORTED, "at most %d electrodes for constrained charges", CCM_MAXE);
  double sum = 0.0, asum = 0.0;
  for (int a = 0; a < ne; ++a) {
    if (!std::isfinite(h_Q[a])) return fail(c, CPM_EINVAL, "charge target %d not finite", a);
    sum += h_Q[a];
    asum += std::fabs(h_Q[a]);
  }
  if (std::fabs(sum) > 1e-12 * std::max(asum, 1e-300))
    return fail(c, CPM_EINVAL, "electrode charge targets must sum to zero (sum = %g)", sum);
  Buffers& b = c->b;
  TRY(dalloc(c, &b.ccmU, (size_t)c->npad * ne));
  TRY(dalloc(c, &b.ccmC, (size_t)ne * ne + ne));
  launch_ccm_response(c->stream, n, c->npad, b.Ainv, b.eid, ne, b.ccmU);
  TRY(launched(c, "ccm response"));
  std::vector<double> U((size_t)n * ne);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(U.data(), b.ccmU, U.size() * sizeof(double), hipMemcpyDeviceToHost));
  // C~ = G^T A^-1 G, then its inverse by Gauss-Jordan with partial pivoting
  std::vector<double> M((size_t)ne * 2 * ne, 0.0);
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < ne; ++a) M[(size_t)c->h_eid[i] * 2 * ne + a] += U[(size_t)i * ne + a];
  for (int a = 0; a < ne; ++a) M[(size_t)a * 2 * ne + ne + a] = 1.0;
  for (int col = 0; col < ne; ++col) {
    int piv = col;
    for (int r = col + 1; r < ne; ++r)
      if (std::fabs(M[(size_t)r * 2 * ne + col]) > std::fabs(M[(size_t)piv * 2 * ne + col])) piv = r;
    if (!(std::fabs(M[(size_t)piv * 2 * ne + col]) > 0.0))
      return fail(c, CPM_ENOTPD, "electrode capacitance matrix is singular");
    if (piv != col)
      for (int k = 0; k < 2 * ne; ++k) std::swap(M[(size_t)col * 2 * ne + k], M[(size_t)piv * 2 * ne + k]);
    const double d = M[(size_t)col * 2 * ne + col];
    for (int k = 0; k < 2 * ne; ++k) M[(size_t)col * 2 * ne + k] /= d;
    for (int r = 0; r < ne; ++r) {
      if (r == col) continue;
      const double f = M[(size_t)r * 2 * ne + col];
      for (int k = 0; k < 2 * ne; ++k) M[(size_t)r * 2 * ne + k] -= f * M[(size_t)col * 2 * ne + k];
    }
  }
  std::vector<double> h((size_t)ne * ne + ne);
  for (int a = 0; a < ne; ++a)
    for (int k = 0; k < ne; ++k) h[(size_t)a * ne + k] = M[(size_t)a * 2 * ne + ne + k];
  for (int a = 0; a < ne; ++a) h[(size_t)ne * ne + a] = h_Q[a];
  HIP_TRY(c, hipMemcpy(b.ccmC, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
  c->have_q = true;
  return CPM_OK;
}

cpm_status cpm_autotune(cpm_ctx* c, int batch, int reps) {
  if (!c) return CPM_EINVAL;
  TRY(finish_invert(c));
  if (!c->have_inv || c->factor_only || !(c->store & CPM_STORE_BF16X2) || !c->b.Shi)
    return fail(c, CPM_ESTATE, "cpm_autotune needs cpm_invert with the split-BF16 copy of S");
  if (batch <= 0 || reps <= 0) return fail(c, CPM_EINVAL, "need batch > 0 and reps > 0");
  const int rows = ((batch + TILE - 1) / TILE) * TILE, npad = c->npad;
  TRY(ensure_solve_buffers(c, rows));
  TRY(ensure_kpart(c, (size_t)4 * rows * npad));
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  cpm_ctx::GemmCfg best;
  best.us = 1e300;
  for (int bm : {32, 64, 128}) {
    if (rows % bm) continue;
    for (int ks : {1, 2, 4}) {
      const int total = rows / bm * (npad / 64) * ks;
      std::vector<int> grids{total};
      for (int g : {256, 512, 1024})
        if (g < total) grids.push_back(g);
      for (int grid : grids) {
        cpm_ctx::GemmCfg cfg;
        cfg.bm = bm; cfg.ks = ks; cfg.grid = grid;
        enqueue_bf16(c, c->b.bpad, c->b.qt, rows, false, cfg, ctx_work(c));    // warm-up
        HIP_TRY(c, hipEventRecord(e0, c->stream));
        for (int r = 0; r < reps; ++r) enqueue_bf16(c, c->b.bpad, c->b.qt, rows, false, cfg, ctx_work(c));
        HIP_TRY(c, hipEventRecord(e1, c->stream));
        TRY(launched(c, "autotune"));
        HIP_TRY(c, hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
        cfg.us = 1e3 * ms / reps;
        if (cfg.us < best.us) best = cfg;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tuned[rows] = best;
  c->last_tune = best;
  return CPM_OK;
}

}  // extern "C"

namespace {

// validation and (first-use) allocation of a grouped solve
cpm_status grouped_prepare(cpm_ctx* const* ctxs, int n_ctx, const int* batch,
                           const void* const* d_b, int b_is_f32, unsigned mode,
                           double* const* d_q) {
  if (!ctxs || n_ctx <= 0 || !batch || !d_b || !d_q) return CPM_EINVAL;
  cpm_ctx* c0 = ctxs[0];
  if (!c0) return CPM_EINVAL;
  if (n_ctx > GB_MAXP) return fail(c0, CPM_EINVAL, "at most %d contexts per group", GB_MAXP);
  if ((mode & 0xffu) != CPM_SOLVE_BF16X2 || (mode & ~0x1ffu))
    return fail(c0, CPM_EUNSUPPORTED, "grouped solves run the split-BF16 mode (0x2 or 0x102)");
  for (int i = 0; i < n_ctx; ++i) {
    if (!ctxs[i]) return fail(c0, CPM_EINVAL, "context %d is NULL", i);
    if (ctxs[i]->stream != c0->stream)
      return fail(c0, CPM_EINVAL, "grouped contexts must share one stream");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(c0, CPM_EINVAL, "context %d appears twice", i);
    TRY(sc_prepare(ctxs[i], batch[i], d_b[i], b_is_f32, mode, d_q[i]));
  }
  return CPM_OK;
}

// the launches of a grouped solve (no allocation, copy or memset)
cpm_status grouped_enqueue(cpm_ctx* const* ctxs, int n_ctx, const int* batch,
                           const void* const* d_b, int b_is_f32, unsigned mode,
                           double* const* d_q, double* const* d_Qe) {
  cpm_ctx* c0 = ctxs[0];
  const bool refine = (mode & CPM_SOLVE_REFINE) != 0;
  hipStream_t st = c0->stream;
  // one persistent launch of S~ products over every context's tiles
  auto group_apply = [&](bool second) {
    GemmGroupBf grp{};
    grp.nprob = n_ctx;
    for (int i = 0; i < n_ctx; ++i) {
      cpm_ctx* c = ctxs[i];
      const int rows = ((batch[i] + TILE - 1) / TILE) * TILE;
      launch_split_bf16(st, (size_t)rows * c->npad, second ? c->b.res : c->b.bpad, c->b.xhi,
                        c->b.xlo);
      grp.p[i] = gemm_bf16x3_problem(rows, c->npad, c->npad, c->b.xhi, c->b.xlo, c->npad,
                                     c->b.Shi, c->b.Slo, c->npad, second ? c->b.qt : c->b.qpad,
                                     c->npad, second ? 1 : 0, 64, 1, nullptr);
    }
    group_finish(grp);
    Timed t(c0, "gemm_bf16x3_grouped");
    launch_gemm_bf16x3_group(st, grp, 64, std::min(grp.total, 1024));
  };
  for (int i = 0; i < n_ctx; ++i) {
    cpm_ctx* c = ctxs[i];
    launch_row_means(st, c->n, batch[i], d_b[i], b_is_f32, c->n, c->b.means);
    launch_pad_rows(st, c->n, c->npad, batch[i], ((batch[i] + TILE - 1) / TILE) * TILE, d_b[i],
                    b_is_f32, c->b.means, c->b.bpad);
  }
  group_apply(false);
  for (int i = 0; i < n_ctx; ++i) {
    cpm_ctx* c = ctxs[i];
    Buffers& b = c->b;
    const int n = c->n, npad = c->npad, rows = ((batch[i] + TILE - 1) / TILE) * TILE;
    double* Qe = d_Qe ? d_Qe[i] : nullptr;
    if (!refine) {
      launch_finalize(st, n, batch[i], b.qpad, npad, b.d, b.u, b.scal, b.eid, c->n_e, d_q[i], n, Qe);
      continue;
    }
    launch_finalize(st, n, batch[i], b.qpad, npad, b.d, b.u, b.scal, b.eid, c->n_e, b.qt, npad,
                    nullptr);
    launch_make_rhs(st, n, npad, batch[i], d_b[i], b_is_f32, b.vat, b.res);
    launch_gemm_f64(st, false, false, rows, npad, npad, -1.0, b.qt, npad, b.A, npad, 1.0, b.res,
                    npad, 0, 0);
    launch_center_rows(st, n, npad, batch[i], b.res);
  }
  if (refine) {
    group_apply(true);
    for (int i = 0; i < n_ctx; ++i) {
      cpm_ctx* c = ctxs[i];
      launch_finalize(st, c->n, batch[i], c->b.qt, c->npad, nullptr, c->b.u, c->b.scal, c->b.eid,
                      c->n_e, d_q[i], c->n, d_Qe ? d_Qe[i] : nullptr);
    }
  }
  return launched(c0, "grouped solve");
}

}  // namespace

extern "C" {

cpm_status cpm_solve_grouped(cpm_ctx* const* ctxs, int n_ctx, const int* batch,
                             const void* const* d_b, int b_is_f32, unsigned mode,
                             double* const* d_q, double* const* d_Qe) {
  if (!ctxs || n_ctx <= 0 || !batch || !d_b || !d_q) return CPM_EINVAL;
  TRY(grouped_prepare(ctxs, n_ctx, batch, d_b, b_is_f32, mode, d_q));
  return grouped_enqueue(ctxs, n_ctx, batch, d_b, b_is_f32, mode, d_q, d_Qe);
}

cpm_status cpm_capture_grouped(cpm_ctx* const* ctxs, int n_ctx, const int* batch,
                               const double* const* d_xyz, void* const* d_b, int b_is_f32,
                               unsigned mode, double* const* d_q, double* const* d_Qe) {
  if (!ctxs || n_ctx <= 0 || !batch || !d_xyz || !d_b || !d_q || !ctxs[0]) return CPM_EINVAL;
  cpm_ctx* c0 = ctxs[0];
  if (!c0->stream)
    return fail(c0, CPM_EINVAL, "graph capture needs a non-default stream for the contexts");
  for (int i = 0; i < n_ctx; ++i) {
    if (!ctxs[i]) return fail(c0, CPM_EINVAL, "context %d is NULL", i);
    TRY(pv_prepare(ctxs[i], batch[i], d_xyz[i], d_b[i], b_is_f32));
  }
  TRY(grouped_prepare(ctxs, n_ctx, batch, d_b, b_is_f32, mode, d_q));
  HIP_TRY(c0, hipStreamSynchronize(c0->stream));
  if (c0->ggraph_exec) { (void)hipGraphExecDestroy(c0->ggraph_exec); c0->ggraph_exec = nullptr; }
  if (c0->ggraph) { (void)hipGraphDestroy(c0->ggraph); c0->ggraph = nullptr; }
  c0->ggroup.clear();
  std::vector<char> timing(n_ctx);
  for (int i = 0; i < n_ctx; ++i) {
    timing[i] = ctxs[i]->timing;
    ctxs[i]->timing = false;                       // no event nodes in the graph
    ctxs[i]->capturing = true;                     // one stream in the graph
  }
  cpm_status st = CPM_OK;
  const hipError_t eb = hipStreamBeginCapture(c0->stream, hipStreamCaptureModeThreadLocal);
  if (eb != hipSuccess) st = fail(c0, CPM_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(eb));
  for (int i = 0; i < n_ctx && st == CPM_OK && eb == hipSuccess; ++i)
    st = pv_enqueue(ctxs[i], batch[i], d_xyz[i], d_b[i], b_is_f32);
  if (st == CPM_OK) st = grouped_enqueue(ctxs, n_ctx, batch, d_b, b_is_f32, mode, d_q, d_Qe);
  hipGraph_t g = nullptr;
  const hipError_t e = eb == hipSuccess ? hipStreamEndCapture(c0->stream, &g) : eb;
  for (int i = 0; i < n_ctx; ++i) {
    ctxs[i]->timing = timing[i] != 0;
    ctxs[i]->capturing = false;
  }
  if (st != CPM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(c0, CPM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  c0->ggraph = g;
  HIP_TRY(c0, hipGraphInstantiate(&c0->ggraph_exec, c0->ggraph, nullptr, nullptr, 0));
  for (int i = 0; i < n_ctx; ++i) c0->ggroup.push_back({ctxs[i], ctxs[i]->alloc_gen});
  return CPM_OK;
}

cpm_status cpm_replay_grouped(cpm_ctx* const* ctxs, int n_ctx) {
  if (!ctxs || n_ctx <= 0 || !ctxs[0]) return CPM_EINVAL;
  cpm_ctx* c0 = ctxs[0];
  if (!c0->ggraph_exec) return fail(c0, CPM_ESTATE, "cpm_replay_grouped before cpm_capture_grouped");
  if ((int)c0->ggroup.size() != n_ctx)
    return fail(c0, CPM_EINVAL, "the group differs from the captured one");
  for (int i = 0; i < n_ctx; ++i) {
    cpm_ctx* c = ctxs[i];
    if (c != c0->ggroup[i].first) return fail(c0, CPM_EINVAL, "context %d differs from the capture", i);
    TRY(finish_invert(c));
    // the graph holds raw device addresses of every context's buffers
    if (c->alloc_gen != c0->ggroup[i].second || !c->have_inv || c->factor_only || !c->have_v ||
        !(c->store & CPM_STORE_BF16X2))
      return fail(c0, CPM_ESTATE, "context %d changed since cpm_capture_grouped; capture again", i);
  }
  HIP_TRY(c0, hipGraphLaunch(c0->ggraph_exec, c0->stream));
  return CPM_OK;
}

cpm_status cpm_enable_timing(cpm_ctx* c, const char* families) {
  if (!c) return CPM_EINVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  resolve_timing(c, true);
  c->totals.clear();
  c->timing_only.clear();
  c->timing = families && families[0];
  if (c->timing && std::strcmp(families, "*") != 0) {
    std::string cur;
    for (const char* p = families;; ++p) {
      if (*p == ',' || *p == 0) {
        if (!cur.empty()) c->timing_only.push_back(cur);
        cur.clear();
        if (*p == 0) break;
      } else if (*p != ' ') {
        cur.push_back(*p);
      }
    }
  }
  return CPM_OK;
}

cpm_status cpm_get_timing(cpm_ctx* c, const char* name, double* total_ms, long long* count) {
  if (!c || !name || !total_ms || !count) return CPM_EINVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  resolve_timing(c, true);
  auto it = c->totals.find(name);
  *total_ms = (it == c->totals.end()) ? 0.0 : it->second.first;
  *count = (it == c->totals.end()) ? 0 : it->second.second;
  return CPM_OK;
}

cpm_status cpm_apply_elastance(cpm_ctx* c, int batch, const double* d_x, double* d_y) {
  if (!c) return CPM_EINVAL;
  if (!c->have_op && !c->have_A)
    return fail(c, CPM_ESTATE, "cpm_apply_elastance needs cpm_build_operator or cpm_build_elastance");
  TRY(wait_invert(c));                    // A may be assembled on the inversion's stream
  TRY(assemble_A(c, c->stream));
  if (batch < 0 || (batch > 0 && (!d_x || !d_y)))
    return fail(c, CPM_EINVAL, "need batch >= 0 and non-NULL d_x, d_y");
  if (batch == 0) return CPM_OK;
  TRY(ensure_cg_buffers(c));
  Buffers& b = c->b;
  hipStream_t st = c->stream;
  const int n = c->n, nslot = cg_nslot(c), nb = cg_grid(c);
  double* P = b.cgv + (size_t)2 * CG_MAXG * nslot;
  double* AP = P + (size_t)CG_MAXG * nslot;
  for (int v0 = 0; v0 < batch; v0 += CG_MAXG) {
    const int g = std::min(CG_MAXG, batch - v0);
    launch_cg_gather(st, nb, nslot, n, g, cg_slots(c), b, d_x + (size_t)v0 * n, P, b.cgred);
    apply_A(c, P, AP, false);
    launch_cg_scatter(st, nb, nslot, n, g, cg_slots(c), AP, d_y + (size_t)v0 * n);
    TRY(launched(c, "apply elastance"));
  }
  return CPM_OK;
}

// cpm_solve_cg is synchronous, so a context on the default (NULL) stream can
// run it on an internal stream, where its iteration blocks can be captured as
// graphs: the NULL stream is drained first, and the internal stream is drained
// and the context's stream restored on every return.
struct CgStream {
  cpm_ctx* c;
  hipStream_t saved;
  bool on = false;
  ~CgStream() {
    if (!on) return;
    (void)hipStreamSynchronize(c->stream);
    c->stream = saved;
  }
};

cpm_status cpm_solve_cg(cpm_ctx* c, int batch, const void* d_b, int b_is_f32, double tol,
                        int maxit, double* d_q, double* d_Qe) {
  if (!c) return CPM_EINVAL;
  if (!c->have_op && !c->have_A)
    return fail(c, CPM_ESTATE, "cpm_solve_cg needs cpm_build_operator or cpm_build_elastance");
  TRY(wait_invert(c));                    // A may be assembled on the inversion's stream
  TRY(assemble_A(c, c->stream));
  if (!c->have_v) return fail(c, CPM_ESTATE, "cpm_solve_cg before cpm_set_potential");
  if (batch < 0 || (batch > 0 && (!d_b || !d_q)))
    return fail(c, CPM_EINVAL, "need batch >= 0 and non-NULL d_b, d_q");
  if (b_is_f32 != 0 && b_is_f32 != 1) return fail(c, CPM_EINVAL, "b_is_f32 must be 0 or 1");
  if (!std::isfinite(tol) || tol < 0.0 || maxit < 1)
    return fail(c, CPM_EINVAL, "need a finite tol >= 0 and maxit >= 1");
  c->cg_iters = 0;
  c->cg_resid = 0.0;
  if (batch == 0) return CPM_OK;
  CgStream swap{c, c->stream};
  if (!c->stream && c->cg_graphs && !c->timing) {
    if (!c->cg_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cg_stream, hipStreamNonBlocking));
    HIP_TRY(c, hipStreamSynchronize(nullptr));
    c->stream = c->cg_stream;
    swap.on = true;
  }
  TRY(ensure_cg_buffers(c));
  TRY(ensure_precond(c));
  Buffers& b = c->b;
  hipStream_t st = c->stream;
  const int n = c->n, nslot = cg_nslot(c), nb = cg_grid(c);
  const int npc = c->pc_tiles;            // 0: plain CG
  const int* slots = cg_slots(c);
  double* X = b.cgv;
  double* R = X + (size_t)CG_MAXG * nslot;
  double* P = R + (size_t)CG_MAXG * nslot;
  double* AP = P + (size_t)CG_MAXG * nslot;
  const double tol2 = tol * tol;
  const size_t bsz = b_is_f32 ? sizeof(float) : sizeof(double);
  const int row_rr = cg_scalar_row(0), row_rr0 = cg_scalar_row(1), row_it = cg_scalar_row(2);
  std::vector<double> h_scal((size_t)CG_NSCAL * CG_MAXG);
  bool all_conv = true;
  for (int v0 = 0; v0 < batch; v0 += CG_MAXG) {
    const int g = std::min(CG_MAXG, batch - v0);
    const void* bsrc = static_cast<const char*>(d_b) + (size_t)v0 * n * bsz;
    { Timed t(c, "cg_init");
      launch_cg_init(st, nb, nslot, n, g, slots, b, bsrc, b_is_f32, X, R, P, b.cgred, b.cgscal);
      if (npc > 0) {       // p = z - mean z, z = M^-1 r0 (r.z into the parity-0 field)
        precond_apply(c, 0, R, AP);
        launch_cg_dir(st, nb, nslot, n, 1, tol2, npc, 1, slots, b, R, AP, P, b.cgred, b.cgscal);
      } }
    TRY(launched(c, "cg init"));
    int it = 0;
    bool conv = false;
    auto iteration = [&](int cur) {
      apply_A(c, P, AP, true);
      { Timed t(c, "cg_update");
        launch_cg_update(st, nb, nslot, n, cur, tol2, npc, slots, X, R, P, AP, b.cgred,
                         b.cgscal); }
      if (npc > 0) {       // z = M^-1 r into AP (free until the next product)
        Timed t(c, "cg_precond");
        precond_apply(c, 1 - cur, R, AP);
      }
      { Timed t(c, "cg_dir");
        launch_cg_dir(st, nb, nslot, n, cur, tol2, npc, 0, slots, b, R, AP, P, b.cgred,
                      b.cgscal); }
    };
    while (it < maxit && !conv) {
      // a block of iterations between convergence checks; vectors below the
      // tolerance are frozen (zero step) by the step-length kernel.  A full
      // block (it even) replays one captured graph of its 8 iterations when
      // the context has its own stream and timing is off.
      const int blk = std::min(8, maxit - it);
      // (re)capture the block's graph when stale; a capture or instantiation
      // that fails turns the graphs off for this context (nothing captured
      // has run), and the block runs eagerly
      auto capture = [&]() {
        if (c->cg_graph_exec) { (void)hipGraphExecDestroy(c->cg_graph_exec); c->cg_graph_exec = nullptr; }
        if (c->cg_graph) { (void)hipGraphDestroy(c->cg_graph); c->cg_graph = nullptr; }
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
          (void)hipGetLastError();
          return false;
        }
        for (int k = 0; k < 8; ++k) iteration(k & 1);
        hipGraph_t gr = nullptr;
        if (hipStreamEndCapture(st, &gr) != hipSuccess || !gr ||
            hipGraphInstantiate(&c->cg_graph_exec, gr, nullptr, nullptr, 0) != hipSuccess) {
          (void)hipGetLastError();
          if (gr) (void)hipGraphDestroy(gr);
          c->cg_graph_exec = nullptr;
          return false;
        }
        c->cg_graph = gr;
        c->cg_graph_gen = c->alloc_gen;
        c->cg_graph_tol2 = tol2;
        c->cg_graph_npc = npc;
        return true;
      };
      bool use_graph = blk == 8 && c->cg_graphs && st && !c->timing;
      if (use_graph && !(c->cg_graph_exec && c->cg_graph_gen == c->alloc_gen &&
                         c->cg_graph_tol2 == tol2 && c->cg_graph_npc == npc))
        use_graph = c->cg_graphs = capture();
      if (use_graph) {
        HIP_TRY(c, hipGraphLaunch(c->cg_graph_exec, st));
        it += 8;
      } else {
        for (int k = 0; k < blk; ++k, ++it) iteration(it & 1);
      }
      TRY(launched(c, "cg iterations"));
      HIP_TRY(c, hipMemcpyAsync(h_scal.data(), b.cgscal, h_scal.size() * sizeof(double),
                                hipMemcpyDeviceToHost, st));
      HIP_TRY(c, hipStreamSynchronize(st));
      conv = true;
      for (int s = 0; s < g; ++s)
        if (!(h_scal[(size_t)row_rr * CG_MAXG + s] <= tol2 * h_scal[(size_t)row_rr0 * CG_MAXG + s]))
          conv = false;
    }
    for (int s = 0; s < g; ++s) {
      const double rr = h_scal[(size_t)row_rr * CG_MAXG + s], rr0 = h_scal[(size_t)row_rr0 * CG_MAXG + s];
      c->cg_iters = std::max(c->cg_iters, (int)h_scal[(size_t)row_it * CG_MAXG + s]);
      const double rel = rr0 > 0.0 ? std::sqrt(rr / rr0) : (rr > 0.0 ? INFINITY : 0.0);
      c->cg_resid = std::max(c->cg_resid, std::isnan(rel) ? INFINITY : rel);
    }
    all_conv = all_conv && conv;
    { Timed t(c, "cg_finish");
      launch_cg_finish(st, nb, nslot, n, g, slots, X, b.cgred, b.eid, c->n_e,
                       d_q + (size_t)v0 * n, d_Qe ? d_Qe + (size_t)v0 * c->n_e : nullptr); }
    TRY(launched(c, "cg finish"));
  }
  HIP_TRY(c, hipStreamSynchronize(st));
  if (!all_conv)
    return fail(c, CPM_ENOCONV, "conjugate gradients stopped at %d iterations with relative residual %g > %g",
                maxit, c->cg_resid, tol);
  return CPM_OK;
}

}  // extern "C"

namespace {

// ---- state files (cpm_save / cpm_load) -------------------------------------
// A 256-byte little-endian header, the matrices as n x n row-major FP64 (A,
// then A^-1 when present), and a trailing 64-bit checksum (FNV-1a over the
// payload's 64-bit words).
constexpr char FILE_MAGIC[8] = {'C', 'P', 'M', 'S', 'T', 'A', 'T', 'E'};
constexpr uint32_t FILE_VERSION = 1;
constexpr size_t FILE_HEADER = 256;

struct FileHeader {
  char magic[8];
  uint32_t version, header_bytes;
  int32_t n, n_e;
  uint32_t matrices, store;
  uint64_t geom_hash;
  double s_sum;
  double knobs[12];               // Lx Ly h slab_factor eta alpha rcut kspace_eps kcut k_e Lz k_c
  int32_t geometry, pad;
  uint64_t payload_bytes;
  unsigned char reserved[88];
  uint64_t header_check;          // FNV-1a of the 248 bytes before it
};
static_assert(sizeof(FileHeader) == FILE_HEADER, "state file header layout");

uint64_t fnv1a_words(uint64_t h, const double* v, size_t count) {
  for (size_t i = 0; i < count; ++i) {
    uint64_t w;
    std::memcpy(&w, v + i, 8);
    h ^= w;
    h *= 1099511628211ull;
  }
  return h;
}

// read and check a header; on success the file is positioned at the payload
cpm_status read_header(FILE* f, FileHeader& hd, std::string& why) {
  if (std::fread(&hd, 1, FILE_HEADER, f) != FILE_HEADER) { why = "file shorter than its header"; return CPM_EINVAL; }
  if (std::memcmp(hd.magic, FILE_MAGIC, 8) != 0) { why = "not a cpm state file (magic)"; return CPM_EINVAL; }
  if (hd.version != FILE_VERSION || hd.header_bytes != FILE_HEADER) {
    why = "unsupported state file version";
    return CPM_EINVAL;
  }
  if (fnv1a(1469598103934665603ull, &hd, FILE_HEADER - 8) != hd.header_check) {
    why = "header checksum mismatch";
    return CPM_EINVAL;
  }
  if (hd.n <= 0 || hd.n_e <= 0 || hd.n_e > hd.n || (hd.matrices != 1 && hd.matrices != 2) ||
      hd.payload_bytes != (uint64_t)hd.matrices * hd.n * hd.n * sizeof(double)) {
    why = "inconsistent sizes in the header";
    return CPM_EINVAL;
  }
  const long pos = std::ftell(f);
  if (std::fseek(f, 0, SEEK_END) != 0) { why = "cannot seek"; return CPM_EINVAL; }
  const long end = std::ftell(f);
  if (end < 0 || (uint64_t)end != FILE_HEADER + hd.payload_bytes + 8) {
    why = "file length does not match the header (truncated or extended)";
    return CPM_EINVAL;
  }
  std::fseek(f, pos, SEEK_SET);
  return CPM_OK;
}

struct FileCloser {
  FILE* f;
  ~FileCloser() { if (f) std::fclose(f); }
};

}  // namespace

extern "C" {

cpm_status cpm_inspect_file(const char* path, cpm_file_info* out) {
  if (!path || !out) return CPM_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) return CPM_EINVAL;
  FileCloser fc{f};
  FileHeader hd;
  std::string why;
  const cpm_status st = read_header(f, hd, why);
  if (st != CPM_OK) return st;
  std::memset(out, 0, sizeof *out);
  out->n = hd.n;
  out->n_e = hd.n_e;
  out->matrices = (int)hd.matrices;
  out->store = hd.store;
  out->geometry_hash = hd.geom_hash;
  out->s_sum = hd.s_sum;
  cpm_params& p = out->params;
  p.Lx = hd.knobs[0]; p.Ly = hd.knobs[1]; p.h = hd.knobs[2]; p.slab_factor = hd.knobs[3];
  p.eta = hd.knobs[4]; p.alpha = hd.knobs[5]; p.rcut = hd.knobs[6]; p.kspace_eps = hd.knobs[7];
  p.kcut = hd.knobs[8]; p.coulomb_k = hd.knobs[9]; p.geometry = hd.geometry;
  return CPM_OK;
}

cpm_status cpm_save(const cpm_ctx* cc, const char* path) {
  if (!cc) return CPM_EINVAL;
  cpm_ctx* c = const_cast<cpm_ctx*>(cc);
  if (!path) return fail(c, CPM_EINVAL, "path is NULL");
  TRY(finish_invert(c));
  if (!c->have_A) return fail(c, CPM_ESTATE, "cpm_save needs cpm_build_elastance");
  TRY(assemble_A(c, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int n = c->n, npad = c->npad;
  FileHeader hd;
  std::memset(&hd, 0, sizeof hd);
  std::memcpy(hd.magic, FILE_MAGIC, 8);
  hd.version = FILE_VERSION;
  hd.header_bytes = FILE_HEADER;
  hd.n = n;
  hd.n_e = c->n_e;
  hd.matrices = (c->have_inv && !c->factor_only) ? 2 : 1;   // A^-1 only when it was formed
  hd.store = c->have_inv ? c->store : 0;
  hd.geom_hash = c->geom_hash;
  hd.s_sum = c->have_inv ? c->s_sum : 0.0;
  const cpm_params& p = c->p;
  const double knobs[12] = {p.Lx, p.Ly, p.h, p.slab_factor, p.eta, p.alpha, p.rcut,
                            p.kspace_eps, p.kcut, c->ke, c->Lz, c->kc};
  std::memcpy(hd.knobs, knobs, sizeof knobs);
  hd.geometry = p.geometry;
  hd.payload_bytes = (uint64_t)hd.matrices * n * n * sizeof(double);
  hd.header_check = fnv1a(1469598103934665603ull, &hd, FILE_HEADER - 8);
  // written to a temporary name, renamed when complete
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return fail(c, CPM_EINVAL, "cannot open %s for writing", tmp.c_str());
  cpm_status st = CPM_OK;
  {
    FileCloser fc{f};
    if (std::fwrite(&hd, 1, FILE_HEADER, f) != FILE_HEADER)
      st = fail(c, CPM_EINVAL, "write of %s failed", tmp.c_str());
    const size_t rows = std::max<size_t>(1, ((size_t)8 << 20) / n);   // 64 MB chunks
    std::vector<double> buf(rows * n);
    uint64_t chk = 1469598103934665603ull;
    const double* mats[2] = {c->b.A, c->b.Ainv};
    for (uint32_t mi = 0; mi < hd.matrices && st == CPM_OK; ++mi)
      for (size_t r0 = 0; r0 < (size_t)n && st == CPM_OK; r0 += rows) {
        const size_t nr = std::min(rows, (size_t)n - r0);
        if (hipMemcpy2D(buf.data(), n * sizeof(double), mats[mi] + r0 * npad, npad * sizeof(double),
                        n * sizeof(double), nr, hipMemcpyDeviceToHost) != hipSuccess) {
          st = fail(c, CPM_EHIP, "device-to-host copy for cpm_save failed");
          break;
        }
        chk = fnv1a_words(chk, buf.data(), nr * n);
        if (std::fwrite(buf.data(), sizeof(double), nr * n, f) != nr * n)
          st = fail(c, CPM_EINVAL, "write of %s failed", tmp.c_str());
      }
    if (st == CPM_OK && std::fwrite(&chk, 1, 8, f) != 8)
      st = fail(c, CPM_EINVAL, "write of %s failed", tmp.c_str());
    if (st == CPM_OK && std::fflush(f) != 0) st = fail(c, CPM_EINVAL, "write of %s failed", tmp.c_str());
  }
  if (st != CPM_OK) {
    std::remove(tmp.c_str());
    return st;
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return fail(c, CPM_EINVAL, "cannot rename %s to %s", tmp.c_str(), path);
  }
  return CPM_OK;
}

cpm_status cpm_load(cpm_ctx* c, const char* path) {
  if (!c) return CPM_EINVAL;
  if (!path) return fail(c, CPM_EINVAL, "path is NULL");
  TRY(wait_invert(c));                    // a pending inversion still writes the buffers
  c->inv_failed = false;
  if (!c->have_A || c->have_op)
    return fail(c, CPM_ESTATE, "cpm_load needs cpm_build_elastance (the electrodes) first");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(c, CPM_EINVAL, "cannot open %s", path);
  FileCloser fc{f};
  FileHeader hd;
  std::string why;
  if (read_header(f, hd, why) != CPM_OK) return fail(c, CPM_EINVAL, "%s: %s", path, why.c_str());
  if (hd.n != c->n || hd.n_e != c->n_e)
    return fail(c, CPM_EINVAL, "%s holds n = %d, n_e = %d; the context has n = %d, n_e = %d", path,
                hd.n, hd.n_e, c->n, c->n_e);
  if (hd.geom_hash != c->geom_hash)
    return fail(c, CPM_EINVAL, "%s was saved for other electrodes or parameters (fingerprint mismatch)",
                path);
  const int n = c->n, npad = c->npad;
  Buffers& b = c->b;
  const unsigned store = hd.store & (unsigned)(CPM_STORE_F32 | CPM_STORE_BF16X2);
  if (hd.matrices == 2) TRY(ensure_inverse_buffers(c, store));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->have_inv = c->have_v = c->have_q = false;
  c->A_pending = false;
  // padding rows and columns hold the identity, as after the assembly
  launch_set_identity(c->stream, npad, b.A);
  if (hd.matrices == 2) launch_set_identity(c->stream, npad, b.Ainv);
  TRY(launched(c, "load"));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t rows = std::max<size_t>(1, ((size_t)8 << 20) / n);
  std::vector<double> buf(rows * n);
  uint64_t chk = 1469598103934665603ull;
  double* mats[2] = {b.A, b.Ainv};
  for (uint32_t mi = 0; mi < hd.matrices; ++mi)
    for (size_t r0 = 0; r0 < (size_t)n; r0 += rows) {
      const size_t nr = std::min(rows, (size_t)n - r0);
      if (std::fread(buf.data(), sizeof(double), nr * n, f) != nr * n) {
        c->have_A = false;
        return fail(c, CPM_EINVAL, "%s: short read", path);
      }
      chk = fnv1a_words(chk, buf.data(), nr * n);
      HIP_TRY(c, hipMemcpy2D(mats[mi] + r0 * npad, npad * sizeof(double), buf.data(),
                             n * sizeof(double), n * sizeof(double), nr, hipMemcpyHostToDevice));
    }
  uint64_t stored = 0;
  if (std::fread(&stored, 1, 8, f) != 8 || stored != chk) {
    c->have_A = false;                    // the device copy is not to be trusted
    return fail(c, CPM_EINVAL, "%s: payload checksum mismatch", path);
  }
  if (hd.matrices == 1) return CPM_OK;   // A only: cpm_invert follows
  TRY(form_S(c, c->stream, store));
  HIP_TRY(c, hipMemcpyAsync(&c->s_sum, b.scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (!(std::fabs(c->s_sum - hd.s_sum) <= 1e-12 * std::fabs(hd.s_sum)))
    return fail(c, CPM_EINVAL, "%s: e^T A^-1 e = %.17g differs from the saved %.17g", path, c->s_sum,
                hd.s_sum);
  c->have_inv = true;
  return CPM_OK;
}

cpm_status cpm_copy_matrix(const cpm_ctx* c, int which, double* d_out) {
  if (!c || !d_out) return CPM_EINVAL;
  TRY(finish_invert(const_cast<cpm_ctx*>(c)));
  if (which == 0 && c->have_A) TRY(assemble_A(const_cast<cpm_ctx*>(c), c->stream));
  const double* src = nullptr;
  if (which == 0 && c->have_A) src = c->b.A;
  if (which == 1 && c->have_inv && !c->factor_only) src = c->b.Ainv;
  if (which == 2 && c->have_inv && !c->factor_only) src = c->b.S;
  if (!src) return CPM_ESTATE;
  const int n = c->n, npad = c->npad;
  if (hipMemcpy2DAsync(d_out, n * sizeof(double), src, npad * sizeof(double), n * sizeof(double), n,
                       hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return CPM_EHIP;
  return CPM_OK;
}

cpm_status cpm_copy_vector(const cpm_ctx* c, int which, double* d_out) {
  if (!c || !d_out) return CPM_EINVAL;
  TRY(finish_invert(const_cast<cpm_ctx*>(c)));
  const double* src = nullptr;
  if (which == 0 && c->have_inv) src = c->b.u;
  if (which == 1 && c->have_v && c->have_inv) src = c->b.d;
  if (!src) return CPM_ESTATE;
  if (hipMemcpyAsync(d_out, src, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return CPM_EHIP;
  return CPM_OK;
}

cpm_status cpm_get_info(const cpm_ctx* c, int key, double* out) {
  if (!c || !out) return CPM_EINVAL;
  switch (key) {
    case CPM_INFO_N: *out = c->n; return CPM_OK;
    case CPM_INFO_NK: *out = c->nk; return CPM_OK;
    case CPM_INFO_NE: *out = c->n_e; return CPM_OK;
    case CPM_INFO_S_SUM: {
      const cpm_status st = finish_invert(const_cast<cpm_ctx*>(c));
      *out = c->s_sum;
      return st != CPM_OK ? st : c->have_inv ? CPM_OK : CPM_ESTATE;
    }
    case CPM_INFO_PIVOT: {
      (void)wait_invert(const_cast<cpm_ctx*>(c));
      *out = c->pivot;
      return CPM_OK;
    }
    case CPM_INFO_LZ: *out = c->Lz; return CPM_OK;
    case CPM_INFO_KCUT: *out = c->kc; return CPM_OK;
    case CPM_INFO_M: *out = c->m; return CPM_OK;
    case CPM_INFO_WORKSPACE: *out = (double)c->bytes; return CPM_OK;
    case CPM_INFO_NPAD: *out = c->npad; return CPM_OK;
    case CPM_INFO_NRUNS: *out = c->nruns; return CPM_OK;
    case CPM_INFO_NLAYERS: *out = c->nlayers; return CPM_OK;
    case CPM_INFO_SF_MATRIX: *out = (c->sf_mfma && c->use_sf_mfma) ? 1.0 : 0.0; return CPM_OK;
    case CPM_INFO_TUNE_BM: *out = c->last_tune.bm; return CPM_OK;
    case CPM_INFO_TUNE_KS: *out = c->last_tune.ks; return CPM_OK;
    case CPM_INFO_TUNE_GRID: *out = c->last_tune.grid; return CPM_OK;
    case CPM_INFO_TUNE_US: *out = c->last_tune.us; return CPM_OK;
    case CPM_INFO_GROUP: *out = c->pv_group; return CPM_OK;
    case CPM_INFO_CG_ITERS: *out = c->cg_iters; return CPM_OK;
    case CPM_INFO_CG_RESID: *out = c->cg_resid; return CPM_OK;
    case CPM_INFO_ELL_WIDTH: *out = c->ell_width; return CPM_OK;
    case CPM_INFO_NCOLS: *out = c->ncolsort; return CPM_OK;
    case CPM_INFO_BSR_BLOCKS: *out = c->bsr_blocks; return CPM_OK;
    case CPM_INFO_PC_TILES: *out = c->pc_tiles; return CPM_OK;
    case CPM_INFO_PC_MODE: *out = c->pc_mode; return CPM_OK;
    case CPM_INFO_PC_COARSE: *out = (double)c->pc_tiles * c->pc_kuse; return CPM_OK;
    case CPM_INFO_SF_FP32:
      *out = (c->sf_mfma && c->use_sf_mfma && c->sf32_ok) ? (c->sf16_ok ? 2.0 : 1.0) : 0.0;
      return CPM_OK;
    case CPM_INFO_RS_PLANE: *out = rs_plane(c) ? 1.0 : 0.0; return CPM_OK;
    default: return CPM_EINVAL;
  }
}

cpm_status cpm_synchronize(cpm_ctx* c) {
  if (!c) return CPM_EINVAL;
  TRY(finish_invert(c));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipGetLastError());
  return CPM_OK;
}

const char* cpm_last_error(const cpm_ctx* c) {
  if (!c) return "no context";
  return c->err.c_str();
}

void cpm_destroy(cpm_ctx* c) {
  if (!c) return;
  (void)wait_invert(c);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  if (c->aux_ev) (void)hipEventDestroy(c->aux_ev);
  if (c->ggraph_exec) (void)hipGraphExecDestroy(c->ggraph_exec);
  if (c->ggraph) (void)hipGraphDestroy(c->ggraph);
  if (c->rs_stream) (void)hipStreamDestroy(c->rs_stream);
  if (c->rs_ev_in) (void)hipEventDestroy(c->rs_ev_in);
  if (c->rs_ev_out) (void)hipEventDestroy(c->rs_ev_out);
  if (c->main_ev) (void)hipEventDestroy(c->main_ev);
  if (c->h_async) (void)hipHostFree(c->h_async);
  Buffers& b = c->b;
  dfree(b.ex); dfree(b.ey); dfree(b.ez); dfree(b.efx); dfree(b.efy); dfree(b.efz); dfree(b.eid);
  dfree(b.layer_of); dfree(b.layer_fz); dfree(b.layerT); dfree(b.amap);
  dfree(b.sc_nx); dfree(b.sc_ny); dfree(b.sc_lo); dfree(b.sc_len); dfree(b.sc_koff); dfree(b.sc_n0);
  dfree(b.sc_nidx); dfree(b.tile_nb); dfree(b.sfm_part); dfree(b.sfm_items); dfree(b.sf16_items); dfree(b.sft);
  dfree(b.tile_off); dfree(b.pz); dfree(b.slot_of); dfree(b.b_items); dfree(b.bT); dfree(b.bPhi);
  dfree(b.runs); dfree(b.cols); dfree(b.chunk_col); dfree(b.w2); dfree(b.knx); dfree(b.kny); dfree(b.knz);
  dfree(b.A); dfree(b.L); dfree(b.Dinv); dfree(b.Ainv); dfree(b.S); dfree(b.S32); dfree(b.Shi);
  dfree(b.Slo); dfree(b.u); dfree(b.d); dfree(b.vat); dfree(b.table); dfree(b.elq); dfree(b.flag);
  dfree(b.sf_part); dfree(b.sfw); dfree(b.phik_part); dfree(b.phir_part); dfree(b.dip); dfree(b.qt);
  dfree(b.res); dfree(b.bpad); dfree(b.qpad); dfree(b.scal); dfree(b.means); dfree(b.rtab); dfree(b.ptab);
  dfree(b.xhi); dfree(b.xlo);
  dfree(b.zperm); dfree(b.cq); dfree(b.zr);
  dfree(b.kpart); dfree(b.ccmU); dfree(b.ccmC); dfree(b.sg); dfree(b.zeta); dfree(b.szeta);
  dfree(b.Qpair); dfree(b.ell_col); dfree(b.ell_val); dfree(b.plane_off); dfree(b.dextra);
  dfree(b.bsr_col); dfree(b.bsr_val); dfree(b.cg_items); dfree(b.asmG); dfree(b.asmF);
  dfree(b.Ecat); dfree(b.cg_ident); dfree(b.cgv); dfree(b.cgred);
  dfree(b.cgscal); dfree(b.cgphi); dfree(b.cgY); dfree(b.cgT);
  dfree(b.pc_phi); dfree(b.pc_dinv); dfree(b.pc_C); dfree(b.pc_W); dfree(b.pc_ztr); dfree(b.pc_tplane);
  dfree(b.pc_dblk); dfree(b.pc_daz); dfree(b.pc_H); dfree(b.pc_ypart); dfree(b.pc_y);
  dfree(b.pc_wn); dfree(b.pc_g); dfree(b.pc_cpart);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cg_graph_exec) (void)hipGraphExecDestroy(c->cg_graph_exec);
  if (c->cg_graph) (void)hipGraphDestroy(c->cg_graph);
  if (c->cg_stream) (void)hipStreamDestroy(c->cg_stream);
  for (auto& pe : c->pending) { (void)hipEventDestroy(pe.a); (void)hipEventDestroy(pe.b); }
  for (auto e : c->evpool) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
