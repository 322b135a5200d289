// Library-internal declarations of libcpm (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/cpm.h"

namespace cpm {

constexpr int TILE = 64;           // dense-matrix tile; matrices are padded to it
constexpr int RUN = 16;            // consecutive k_z values per k-space run
constexpr int GEMM_MIN_BATCH = 4;  // batches this large solve as one MFMA GEMM
constexpr double KE_DEFAULT = 14.399645478425668;

// One run of the k-space set: a column (nx, ny) and up to RUN consecutive nz.
struct KRun {
  int nx, ny, nz0, len;
  int koff;                        // index of its first k in the flat k arrays
  int pad;
};

// One column segment of the k-space set: fixed (nx, ny), len consecutive k_z
// starting at lo (at most PJ_MAXK of them).
struct KCol {
  int nx, ny, lo, len;
  int koff;                        // index of its first k in the flat k arrays
  int pad;
};

constexpr int CCM_MAXE = 16;       // electrodes supported by the constrained charge method
constexpr int SFM_NB = 4;          // 16-wide n blocks per matrix-core structure-factor work item
constexpr int SF16_NB = 12;        // ... per item of the split-FP16 kernel (3 per wave)

// charges per chunk of the matrix-core structure factors (a multiple of 16)
inline int sf_mfma_chunk(int mpad, int mchunks) {
  return (((mpad + mchunks - 1) / mchunks) + 15) / 16 * 16;
}

constexpr int RS_NT = 2048;        // intervals of the real-space pair table on [0, rc]
constexpr int RP_N = 512;          // intervals of the planar pair polynomials on [0, rc]
constexpr int RP_DEG = 6;          // their degree in s = r^2
constexpr int RP_REC = 6;          // 8-byte words per interval: a0..a3 FP64, a4..a6 FP32 (48 B)

constexpr int PJ_MAXK = 1024;      // weighted k values staged per projection chunk
constexpr int MAX_LAYERS = 64;     // planar-electrode factorisation up to this many z planes
constexpr int CG_MAXG = 64;        // vectors per conjugate-gradient group (slot-row width)
constexpr int CG_RED = 13;         // block partial fields
constexpr int CG_NSCAL = 4;        // per-vector scalar rows reported to the host

struct Buffers {
  // electrode geometry (internal order = caller order), SoA, x and y wrapped
  double* ex = nullptr;  double* ey = nullptr;  double* ez = nullptr;
  double* efx = nullptr; double* efy = nullptr; double* efz = nullptr;  // fractional
  int* eid = nullptr;
  int* layer_of = nullptr;         // plane index per atom (planar electrodes)
  int* amap = nullptr;             // real-space thread -> atom map: whole waves per plane, -1 pads
  double* layer_fz = nullptr;      // fractional z of each plane
  double2* layerT = nullptr;       // T(column, plane)
  // k-set
  KRun* runs = nullptr;            // nruns
  KCol* cols = nullptr;            // ncols
  int* chunk_col = nullptr;        // kchunks + 1 column boundaries of the projection chunks
  // matrix-core structure factors: full (k_x, k_y) columns sorted by k_z extent
  int* sc_nx = nullptr; int* sc_ny = nullptr; int* sc_lo = nullptr; int* sc_len = nullptr;
  int* sc_koff = nullptr; int* sc_n0 = nullptr; int* sc_nidx = nullptr; int* tile_nb = nullptr;
  double* sfm_part = nullptr;      // chunk partials [chunk][tile][32][npadc]
  int4* sfm_items = nullptr;       // work items {M tile, first n block, n blocks, 0}
  int4* sf16_items = nullptr;      // the same with <= SF16_NB blocks (split-FP16 kernel)
  int* tile_off = nullptr;         // offset of each M tile's block in a chunk of sfm_part
  int* slot_of = nullptr;          // atom -> slot of the atom map (n)
  int* b_items = nullptr;          // work items of the b-path projection product
  double2* pz = nullptr;           // plane phases e^{-i n kz1 z_L} (nlayers x nzt)
  double* bT = nullptr;             // T(c, L) of a group as the projection operand (nL x 2 ncp x 64)
  double* bPhi = nullptr;          // projection parts (b_nparts x slots x 64)
  double2* sft = nullptr;          // per-charge phase tables (rows x mpad)
  double* w2 = nullptr;            // 2 W(k), nk (flat run order)
  int* knx = nullptr; int* kny = nullptr; int* knz = nullptr;     // nk
  // dense matrices, npad x npad row-major FP64 unless noted
  double* A = nullptr;             // elastance (kept for refinement)
  double* L = nullptr;             // work: Cholesky factor, later X = L^-1
  double* Dinv = nullptr;          // nb x 64 x 64 inverses of diagonal blocks of L
  double* Ainv = nullptr;          // A^-1
  double* S = nullptr;             // charge-neutral capacitance (Eq. 4)
  float* S32 = nullptr;            // FP32 copy
  uint16_t* Shi = nullptr;         // split-BF16 copy: S ~ hi + lo
  uint16_t* Slo = nullptr;
  double* u = nullptr;             // A^-1 e (n)
  double* d = nullptr;             // S v (npad)
  double* vat = nullptr;           // per-atom applied potential v = G v~ (npad)
  double* table = nullptr;         // k-space phase table chunk for the A SYRK
  double* asmG = nullptr;          // planar A assembly: G (atom-map rows x 2 columns)
  double* asmF = nullptr;          //   and F^L (2 columns x npad)
  double* elq = nullptr;           // electrolyte charges (m)
  int* flag = nullptr;             // device status word (Cholesky pivot)
  // per-step workspaces
  double* sf_part = nullptr;       // m-chunk partial structure factors (2 * nk * mchunks)
  double* sfw = nullptr;           // 2W-weighted structure factor (2 * nk)
  double* phik_part = nullptr;     // k-chunk partial potentials (n * kchunks)
  double* phir_part = nullptr;     // m-chunk partial real-space potentials (n * rchunks)
  double* dip = nullptr;           // electrolyte dipole partials (per 256 charges, 3 axes)
  double* rtab = nullptr;          // real-space pair table (g, g', g'') x (RS_NT + 1)
  double* ptab = nullptr;          // planar pair polynomials (RP_N x RP_REC), set once
  double* fwork = nullptr;         // factor-only inverse: two 64 x npad right-hand-side blocks
  int* zperm = nullptr;            // order of the charges for the real-space pass (m)
  double4* cq = nullptr;           // gathered charges (x, y wrapped, z, q), pv_group x mpad64
  double2* zr = nullptr;           // z range of each 64-charge block, pv_group x mpad64 / 64
  double* qt = nullptr;            // q-tilde (batch x npad)
  double* res = nullptr;           // refinement residual / corrections (batch x npad)
  double* bpad = nullptr;          // padded b for batched solves (bpad_rows x npad)
  double* qpad = nullptr;          // padded GEMM output (bpad_rows x npad)
  uint16_t* xhi = nullptr;         // left operand of the split-BF16 product, BF16 pairs
  uint16_t* xlo = nullptr;         //   (bpad_rows x npad each)
  double* means = nullptr;         // per-vector uniform part removed before S products
  double* kpart = nullptr;         // split-K partial slices of the batched split-BF16 GEMM
  double* ccmU = nullptr;          // constrained charges: U = A^-1 G (n x n_e)
  double* ccmC = nullptr;          // C~^-1 (n_e x n_e) followed by the targets Q (n_e)
  double* sg = nullptr;            // S G: response of the charges to each electrode's
                                   // potential (npad x n_e, Eq. 6), formed by cpm_invert
  double* zeta = nullptr;          // finite-field zeta (npad, zero padding)
  double* szeta = nullptr;         // S zeta of the finite-field potential (npad)
  // matrix-free operator and conjugate gradients (slot space: the atom map
  // for the operator, atoms padded to npad for the dense A)
  double2* Qpair = nullptr;        // Q_c(L, L') per sorted column, [(c nL + L) nL + L']
  int* ell_col = nullptr;          // real-space + self part of A, ELL rows [slot * width + k]
  double* ell_val = nullptr;       //   (set-up only; kept as 64 x 64 blocks below)
  int* bsr_col = nullptr;          // column tile of each nonzero block (rows of a tile together)
  double* bsr_val = nullptr;       // the blocks, row-major 64 x 64 each
  int* cg_items = nullptr;         // work items of the fused projection / real-space kernel
  int* plane_off = nullptr;        // nlayers + 1 slot offsets of the planes
  double* Ecat = nullptr;          // in-plane phases, (2 ncp) x nslot real matrix
  int* cg_ident = nullptr;         // identity slot map of the dense A (npad, -1 pads)
  double* dextra = nullptr;        // diagonal extra (n)
  double* cgv = nullptr;           // X, R, P, AP: 4 x nslot x CG_MAXG (slot-major)
  double* cgred = nullptr;         // block partials
  double* cgscal = nullptr;        // per-vector r.r, r0.r0, iterations (CG_NSCAL x CG_MAXG)
  double* cgphi = nullptr;         // k- and real-space potentials (nparts x nslot x CG_MAXG)
  double* cgY = nullptr;           // plane sums (ksplit x nlayers x 2 ncp x CG_MAXG)
  double* cgT = nullptr;           // plane-mixed sums (same shape)
  double* pc_dinv = nullptr;       // preconditioner: inverse tile blocks (ntile x 64 x 64)
  double* pc_phi = nullptr;        //   coarse basis functions per slot (nslot x 3)
  double* pc_C = nullptr;          // coarse matrix and its inverse, two ntile x ntile buffers
  double* pc_W = nullptr;
  double* pc_ztr = nullptr;        // tile sums of r (ntile x CG_MAXG)
  int* pc_tplane = nullptr;        // plane of each tile
  int* pc_dblk = nullptr;          // real-space block of each tile's diagonal (-1: none)
  double* pc_daz = nullptr;        // balancing form: B A Z (slots x ld)
  double* pc_H = nullptr;          //   C^-1 + C^-1 (A Z)^T B A Z C^-1 (ld x ld)
  double* pc_ypart = nullptr;      //   parts of (B A Z)^T r (nparts x ld x CG_MAXG)
  double* pc_y = nullptr;          //   their sum, and the coarse vectors w, g (ld x CG_MAXG)
  double* pc_wn = nullptr;
  double* pc_g = nullptr;
  double* pc_cpart = nullptr;      //   parts of the coarse products (cparts x 2 x ld x CG_MAXG)
  size_t kpart_len = 0;
  int bpad_rows = 0;
  double* scal = nullptr;          // small scalars (s and friends)
};

// matrix-free operator and conjugate gradients (cg.hip); vectors are
// slot-major rows of CG_MAXG, slot_atom maps slots to atoms (-1 pads)
int cg_blocks(int nslot, int cap);
int cg_scalar_row(int which);      // 0: r.r, 1: r0.r0, 2: iterations
// real-space + self part of A in ELL form over slots: count per (slot chunk,
// row) cnt[chunk * nslot + r], then fill from offsets off[chunk * nslot + r]
// (entries of a row in ascending slot; padding col = own slot, val = 0)
void launch_ell_count(hipStream_t st, int nslot, int jchunks, const int* slot_atom,
                      const Buffers& b, double Lx, double Ly, double Lz, double rc, int* cnt);
void launch_ell_fill(hipStream_t st, int nslot, int jchunks, int width, const int* slot_atom,
                     const int* off, const Buffers& b, double Lx, double Ly, double Lz, double rc,
                     double alpha, double eta_ee, double diag_self, int* col, double* val);
void launch_cg_ephase(hipStream_t st, int nslot, int ncp, int ncolsort, const int* slot_atom,
                      const Buffers& b, double* Ecat);
// A p on matrix cores: plane sums Y (split over ksplit slot ranges), plane
// mixing T, then the projection and the block-sparse real space per slot
// tile as work items {tile, kind, begin, end, part, plane} into Phi parts
void launch_cg_plane_sums(hipStream_t st, int nslot, int ncp, int nlayers, int ksplit,
                          const int* plane_off, const double* Ecat, const double* P, double* Y);
void launch_cg_plane_mix(hipStream_t st, int ncp, int ncolsort, int nlayers, int ksplit,
                         const double2* Q, const double* Y, double* T);
void launch_cg_tiles(hipStream_t st, int nitems, int nslot, int ncp, const int* items,
                     const double* Ecat, const double* T, const int* bcol, const double* bval,
                     const double* P, double* Phi);
// the b projection for a single configuration (lane 0 of T and Phi), same items
void launch_proj_one(hipStream_t st, int nitems, int nslot, int ncp, const int* items,
                     const double* Ecat, const double* T, double* Phi);
// The kernels below share one grid of nblk blocks; each sums the partials
// of the previous one.  AP (operator; dense: AP given) with partials of p.Ap.
void launch_cg_apply(hipStream_t st, bool dense, int nblk, int nslot, int n, const int* slot_atom,
                     const Buffers& b, int nparts, const double* Phi, double background,
                     const double* cdip, double ke, const double* P, double* AP, double* red);
// x, r update (cur: parity of the iteration; npc > 0: step length from the
// r.z partials of the preconditioner's npc tile blocks), then p and its
// moments (p = z - mean z + beta p with Z = M^-1 r when npc > 0; first: the
// first direction, beta = 0)
void launch_cg_update(hipStream_t st, int nblk, int nslot, int n, int cur, double tol2, int npc,
                      const int* slot_atom, double* X, double* R, const double* P,
                      const double* AP, double* red, double* scal);
void launch_cg_dir(hipStream_t st, int nblk, int nslot, int n, int cur, double tol2, int npc,
                   int first, const int* slot_atom, const Buffers& b, const double* R,
                   const double* Z, double* P, double* red, double* scal);
// two-level preconditioner over the ntile slot tiles: inverses of A's
// 64 x 64 diagonal tile blocks (from the operator's pieces); the coarse
// matrix C = Z^T A Z (Z: K basis functions per tile, phi[slot * 3 + c];
// row stride ld >= ntile K) column block by column block from A applied to
// the basis vectors; C^-1 by Gauss-Jordan steps on the leading block (C and
// W both hold it; returns the one with C^-1).  Per iteration Z = M^-1 R with partials of
// r.z (field of parity `parity`) and of sum z: additive form
// (launch_pc_apply), or balancing form with DAZ = B A Z and H (ld a
// multiple of 64; Ypart: nparts x ld x 64, Y, Tt, Wn, G: ld x 64)
void launch_pc_blocks(hipStream_t st, int ntile, int nslot, int nlayers, int ncolsort,
                      const int* slot_atom, const int* tile_plane, const int* diag_blk,
                      const double* bval, const double* Ecat, const double2* Q, const Buffers& b,
                      double background, const double* cdip, double ke, double* Dinv);
void launch_pc_basis(hipStream_t st, int nblk, int nslot, int K, int j0, int g,
                     const int* slot_atom, const double* phi, const Buffers& b, double* P,
                     double* red);
void launch_pc_coarse_cols(hipStream_t st, int ntile, int ld, int K, int j0, int g,
                           const double* phi, const double* V, double* C);
double* launch_pc_invert(hipStream_t st, int ntile, int ld, double* C, double* W);
void launch_pc_apply(hipStream_t st, int ntile, int ld, int parity, const int* slot_atom,
                     const double* Dinv, const double* Cinv, const double* R, double* Z,
                     double* ZtR, double* red);
void launch_bnn_apply(hipStream_t st, int ntile, int K, int ld, int nparts, int cparts,
                      int parity, const int* slot_atom, const double* phi, const double* Dinv,
                      const double* DAZ, const double* Cinv, const double* H, const double* R,
                      double* Z, double* Ypart, double* Yn, double* Tt, double* Wn, double* G,
                      double* Cpart, double* red);
void launch_cg_init(hipStream_t st, int nblk, int nslot, int n, int g, const int* slot_atom,
                    const Buffers& b, const void* bsrc, int b_is_f32, double* X, double* R,
                    double* P, double* red, double* scal);
void launch_cg_gather(hipStream_t st, int nblk, int nslot, int n, int g, const int* slot_atom,
                      const Buffers& b, const double* x, double* P, double* red);
void launch_cg_scatter(hipStream_t st, int nblk, int nslot, int n, int g, const int* slot_atom,
                       const double* V, double* y);
void launch_cg_finish(hipStream_t st, int nblk, int nslot, int n, int g, const int* slot_atom,
                      const double* X, double* red, const int* eid, int n_e, double* q,
                      double* Qe);

}  // namespace cpm

struct cpm_ctx {
  cpm_params p{};
  hipStream_t stream = nullptr;
  std::string err;
  bool have_elyt = false, have_A = false, have_inv = false, have_v = false, have_q = false;
  bool A_pending = false;          // A's kernels not yet enqueued (done by its first consumer)
  bool A_diag_extra = false;       // a per-atom diagonal term was given (kept in b.dextra)
  bool have_op = false;            // matrix-free operator (cpm_build_operator)
  // cpm_invert with CPM_INVERT_ASYNC: second stream, completion event, pinned
  // host words for s and the pivot flag; joined by the first consumer
  hipStream_t aux = nullptr;
  hipEvent_t aux_ev = nullptr, main_ev = nullptr;
  // real-space pass of cpm_potential_vector on a stream of its own, beside
  // the structure factors (events: inputs ready, real space done)
  hipStream_t rs_stream = nullptr;
  hipEvent_t rs_ev_in = nullptr, rs_ev_out = nullptr;
  bool rs_conc_ok = true;          // CPM_RS_CONCURRENT=0 keeps it on the context stream
  bool capturing = false;          // inside cpm_capture_step (one stream only)
  struct AsyncWords { double s; int flag; };
  AsyncWords* h_async = nullptr;
  bool inv_pending = false, inv_failed = false;
  double op_background = 0.0;      // -pi / (V alpha^2)
  int cg_iters = 0;                // last cpm_solve_cg: iterations, max relative residual
  double cg_resid = 0.0;
  int ell_width = 0;               // entries per row of the real-space ELL part
  int ncp = 0;                     // columns of the operator's k-space products (ncolsort
                                   // rounded up to 32)
  int bsr_blocks = 0;              // nonzero 64 x 64 blocks of the real-space part
  int cg_nitems = 0, cg_nparts = 1, cg_ksplit = 1;   // work split of the operator products
  int n = 0, npad = 0, n_e = 0, m = 0;
  double Lz = 0, V = 0, kc = 0, ke = 0;
  double cdip[3] = {0, 0, 0};      // dipole term A += k_e sum_d cdip_d r_d r_d^T (geometry)
  int dip_blocks = 1;              // electrolyte dipole partials per configuration
  int nk = 0, nruns = 0;
  bool step_ready = false;         // b-path work arrays sized for the current geometry
  int mchunks = 1, kchunks = 1, rchunks = 1;
  int sf_wg_target = 512;          // structure-factor workgroups per snapshot (tuning)
  int sfm_wg_target = 4096;        // the same for the matrix-core kernel
  int sf16_wg_target = 2048;       // ... and for the split-FP16 one
  int sfm_min_chunk = 512;         // fewest charges per matrix-core chunk
  int sfm_max_chunk = 4096;        // most charges per matrix-core chunk
  int chol_block = 512;            // columns per outer block of the Cholesky / inverse (CPM_CHOL_BLOCK)
  int cg_cap = 0;                  // most workgroups of the CG vector kernels (0: by size)
  int cg_precond = 2;              // operator CG preconditioner: 0 none, 1 additive, 2 balancing
  int pc_tiles = 0;                // tiles of the preconditioner in use (0: none or not built)
  int pc_mode = 0;                 // form in use (1 additive, 2 balancing)
  int pc_ld = 0;                   // coarse row stride: coarse columns rounded up to 64
  int pc_k = 0;                    // coarse basis functions per tile (1: constant; 3: + linear;
                                   // 0: by size, 3 from PC_COARSE3_TILES tiles on)
  int pc_kuse = 1;                 // ... in use (the additive form uses 1)
  int pc_nparts = 1;               // slot parts of the balancing form's y product
  int pc_cparts = 1;               // coarse-column parts of its coarse products
  bool pc_ready = false;           // preconditioner built for the current operator
  const double* pc_Cinv = nullptr; // whichever of pc_C / pc_W holds the coarse inverse
  std::vector<int> h_bdiag;        // real-space block of each tile's diagonal (-1: none)
  int rs_wg_target = 0;            // real-space workgroups per launch group (0: by size)
  int rs_sort_min = 16;            // batches of at least this size sort the charges by z
  bool zperm_ok = false;           // b.zperm holds an order of the charges by z
  int pv_fast_min = 1;             // batches from this size take the grouped b path
  unsigned store = 0;
  uint64_t geom_hash = 0;          // fingerprint of A's inputs (cpm_save / cpm_load)
  int field_bottom = -1;           // bottom electrode of the zeta in b.zeta
  bool szeta_ok = false;           // b.szeta = S zeta holds for the current inverse
  double s_sum = 0;                // e^T A^-1 e
  int pivot = -1;
  size_t bytes = 0;
  std::map<const void*, size_t> alloc_sizes;   // device allocations and their sizes
  unsigned long long alloc_gen = 0;    // bumped by every device allocation / free
  std::vector<double> h_v;         // per-electrode potential
  std::vector<double> h_xyz;       // electrode coordinates (host copy)
  std::vector<int> h_eid;
  std::vector<double> h_q;         // electrolyte charges (host copy)
  std::vector<cpm::KRun> h_runs;   // k set, built on the host at create time
  std::vector<cpm::KCol> h_cols;
  std::vector<int> h_chunk_col;
  int nxm = 0, nym = 0, nzm = 0;   // largest |n| per axis in the k set
  int nlayers = 0;                 // > 0: electrodes lie on this many z planes (factorised projection)
  bool sf_mfma = false;            // structure factors on FP64 matrix cores (k set fits)
  bool use_sf_mfma = true;         // tuning switch (CPM_SF_MFMA=0 keeps the VALU kernel)
  bool sf32_ok = true;             // FP32 structure factors when b is stored in FP32
  bool sf16_ok = true;             // ... on FP16 matrix cores with split operands
  int sf16_nt = 2;                 // ... M tiles per work item (1, 2 or 4)
  bool rs_plane_ok = true;         // planar real-space kernel (pair polynomials in r^2)
  bool factor_only = false;        // cpm_invert kept the Cholesky factor, not S
  int ncolsort = 0, sfm_tiles = 0, sfm_npadc = 0, sfm_ntot = 0;
  int sfm_nbz = 2, sfm_nitems = 0, sf16_nitems = 0, mpad = 0, sft_rows = 0, sft_blocks = 1;
  int sfm_pchunk = 0;              // doubles per (configuration, chunk) of sfm_part
  int sfm_maxcnt = 0;              // largest number of n >= 0 of a sorted column
  int pv_group = 1;                // configurations per launch group (planar fast path)
  int pv_group_cap = 64;           // most configurations per launch group (CPM_PV_GROUP)
  int b_nitems = 0, b_nparts = 1;  // work split of the b-path projection product
  int nmap = 0;                    // length of the real-space atom map
  std::vector<int> h_plane_rows;   // rows of the atom map per plane (multiples of 64)
  std::vector<int> h_amap;         // the atom map (host copy)
  std::vector<int> h_tile_plane;   // plane of each 64-slot tile of the atom map
  int planar_nslot = 0;            // slots the planar k-space buffers were sized for
  std::vector<int> h_tile_off;
  std::vector<int4> h_sfm_items, h_sf16_items;
  std::vector<int> h_sc_nx, h_sc_ny, h_sc_lo, h_sc_len, h_sc_koff, h_sc_n0, h_sc_nidx, h_tile_nb;
  std::vector<double> h_w2;
  std::vector<int> h_kx, h_ky, h_kz;
  cpm::Buffers b;
  // split-BF16 batched GEMM configuration per padded row count (cpm_autotune)
  struct GemmCfg { int bm = 64, ks = 1, grid = 0; double us = 0.0; };
  std::map<int, GemmCfg> tuned;
  GemmCfg last_tune;
  // captured step (cpm_capture_step / cpm_replay_step)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  unsigned long long graph_gen = 0;    // alloc_gen when the graph was captured
  // graph of a grouped step (cpm_capture_grouped), held by the first context:
  // the contexts in order with their alloc_gen at capture
  hipGraph_t ggraph = nullptr;
  hipGraphExec_t ggraph_exec = nullptr;
  std::vector<std::pair<cpm_ctx*, unsigned long long>> ggroup;
  // the CG iteration block (8 iterations between convergence checks) as a
  // graph, keyed by the buffers, the tolerance and the preconditioner
  bool cg_graphs = true;
  hipStream_t cg_stream = nullptr;     // internal stream of cpm_solve_cg for the NULL-stream context
  hipGraph_t cg_graph = nullptr;
  hipGraphExec_t cg_graph_exec = nullptr;
  unsigned long long cg_graph_gen = 0;
  double cg_graph_tol2 = -1.0;
  int cg_graph_npc = -1;
  unsigned graph_store = 0;            // copies of S the captured solve reads
  bool graph_ccm = false;              // the captured solve needs the charge targets
  // kernel timing (cpm_enable_timing)
  bool timing = false;
  std::vector<std::string> timing_only;   // empty: every family
  struct Pending { const char* name; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> evpool;
  std::map<std::string, std::pair<double, long long>> totals;
};

namespace cpm {

// ---- launchers (each enqueues on `st`; shapes are checked by the caller) ----
// assembly
void launch_prep_electrodes(hipStream_t st, int n, const double* xyz, double Lx, double Ly,
                            double Lz, Buffers& b);
void launch_real_space_A(hipStream_t st, int n, int npad, const Buffers& b, double Lx, double Ly,
                         double Lz, double rc, double alpha, double eta_ee, double diag_self,
                         double background, const double* cdip, double ke,
                         const double* diag_extra, double* A);
void launch_phase_table(hipStream_t st, int n, int npad, int k0, int kc, int nk, const Buffers& b,
                        double ke, double* table);
void launch_plane_pair_weights(hipStream_t st, int ncolsort, int nlayers, const int* sc_lo,
                                const int* sc_len, const int* sc_koff, const double* w2,
                                const double* layer_fz, double2* Q);
void launch_build_G(hipStream_t st, int nmap, int ncolsort, int ldG, const int* amap,
                    const int* sc_nx, const int* sc_ny, const Buffers& b, double* G);
void launch_build_F(hipStream_t st, int L, int n, int npad, int nlayers, int ncolsort, int ldG,
                    const int* sc_nx, const int* sc_ny, const Buffers& b, const double2* Q,
                    double* F);
void launch_mirror_lower(hipStream_t st, int npad, double* A);

// dense FP64 algebra (MFMA)
// C = beta C + alpha op(A) op(B); M, N multiples of 64; K multiple of 16.
// tri: 0 all tiles, 1 lower tiles only.  kmode: 0 K range [0,K), 1 [max(m0,n0), K).
void launch_gemm_f64(hipStream_t st, bool transA, bool transB, int M, int N, int K,
                     double alpha, const double* A, int lda, const double* B, int ldb,
                     double beta, double* C, int ldc, int tri, int kmode, const int* rowmap = nullptr);
void launch_potrf_diag(hipStream_t st, double* Lblk, int ld, double* Dinv, int* flag, int k0);
void launch_set_identity(hipStream_t st, int npad, double* X);
void launch_row_sums(hipStream_t st, int n, int npad, const double* M, double* out);
void launch_sum_vector(hipStream_t st, int n, const double* v, double* out);
void launch_make_S(hipStream_t st, int n, int npad, const double* Ainv, const double* u,
                   const double* s_dev, double* S);
void launch_convert_S(hipStream_t st, int npad, const double* S, float* S32, uint16_t* hi,
                      uint16_t* lo);

// per-step solve
// y[b] = sign * M x[b] + addscale * add[b * add_ld + .]   (add may be NULL);
// x FP64, npad apart per vector, zero beyond n
void launch_matvec(hipStream_t st, int which /*0 f64, 1 f32*/, int npad, const void* M, int batch,
                   const double* x, const double* add, int add_ld, double addscale, double* y,
                   int ldy, int negate);
// dst[b] (npad apart) = src[b] - (center ? mean_b : 0) for i < n, 0 beyond
void launch_center_pad(hipStream_t st, int n, int npad, int batch, const void* x, int x_is_f32,
                       int ldx, int center, double* dst);
void launch_row_means(hipStream_t st, int n, int batch, const void* x, int x_is_f32, int ldx,
                      double* means);
void launch_center_rows(hipStream_t st, int n, int ld, int batch, double* x);
void launch_make_rhs(hipStream_t st, int n, int npad, int batch, const void* bsrc, int b_is_f32,
                     const double* v, double* c);
// q[b] = (qt[b] + add) - (e^T (qt[b] + add) / s) u ; Qe[b] = G^T q[b]   (add may be NULL)
void launch_finalize(hipStream_t st, int n, int batch, const double* qt, int ldqt, const double* add,
                     const double* u, const double* s_dev, const int* eid, int n_e, double* q,
                     int ldq, double* Qe);
void launch_fill_zero(hipStream_t st, size_t count, float* p);
// U = M G (npad x n_e) in one pass over the symmetric M (n_e <= CCM_MAXE)
void launch_ccm_response(hipStream_t st, int n, int npad, const double* M, const int* eid,
                         int n_e, double* U);
// one value per electrode, passed by value to a kernel
struct ElectrodeValues { double v[CCM_MAXE]; };
void launch_apply_potential(hipStream_t st, int n, int npad, int n_e, const int* eid,
                            const double* SG, const ElectrodeValues& vt, double* vat, double* d);
void launch_scale_field(hipStream_t st, int npad, double dv0, const double* zeta,
                        const double* szeta, double* vat, double* d);
void launch_ccm_finalize(hipStream_t st, int n, int batch, const double* yt, int ldy,
                         const double* U, const double* Cinv, const double* Qt, const int* eid,
                         int n_e, double* q, int ldq, double* Qe);
void launch_pad_rows(hipStream_t st, int n, int npad, int batch, int rows, const void* src,
                     int src_is_f32, const double* shift, double* dst);
// C (M x N, FP64) (+)= Bm (M x K, FP64, split to BF16 hi/lo on load) * S, with
// S symmetric given as BF16 hi/lo (N x K row-major): 3 MFMA products, FP32
// accumulation.  M, N multiples of 64, K multiple of 32.
// split-BF16 GEMM problems, one persistent launch per group (see dense.hip)
constexpr int GB_MAXP = 8;
struct GemmProbBf {
  const uint16_t* Xhi; const uint16_t* Xlo;   // the left operand split into BF16 pairs
  const uint16_t* Shi; const uint16_t* Slo; double* C; double* part;
  int M, N, K, ldx, lds, ldc, tiles_m, tiles_n, ks, accumulate;
};
struct GemmGroupBf {
  int nprob, total;
  int start[GB_MAXP + 1];
  GemmProbBf p[GB_MAXP];
};
GemmProbBf gemm_bf16x3_problem(int M, int N, int K, const uint16_t* Xhi, const uint16_t* Xlo,
                               int ldx, const uint16_t* Shi, const uint16_t* Slo, int lds,
                               double* C, int ldc, int accumulate, int bm, int ks, double* part);
// x ~ hi + lo as BF16 pairs (count FP64 values), the same split as the copies of S
void launch_split_bf16(hipStream_t st, size_t count, const double* x, uint16_t* hi, uint16_t* lo);
void group_finish(GemmGroupBf& grp);
void launch_gemm_bf16x3_group(hipStream_t st, const GemmGroupBf& grp, int bm, int grid);

// b vector
void launch_b_structure_factor(hipStream_t st, int fp32, int nruns, const KRun* runs, int nk,
                               int m, int mchunks, const double* xyz, const double* q,
                               double Lx, double Ly, double Lz, int nxm, int nym, int nzm,
                               double* part);
// per-charge phase tables; fp32: stored as float2 (the same rows, half the bytes)
void launch_b_sf_tables(hipStream_t st, int g, int m, int mpad, int nxm, int nym, int nbz,
                        const double* xyz, const double* q, double Lx, double Ly, double Lz,
                        double2* tab, int fp32, double* dip);
void launch_b_elyt_dipole(hipStream_t st, int g, int m, const double* xyz, const double* q,
                          double* dip);
void launch_dipole_partials(hipStream_t st, int g, int m, const double* xyz, size_t xyz_stride,
                            const double* q, size_t q_stride, double* dip);
// the charges of configuration 0 ordered by z for the real-space pass
void launch_zsort(hipStream_t st, int m, const double* xyz, double Lz, int nbins, int* perm);
int zsort_bins(double Lz);         // z bins of the charge order (about 0.25 A wide)
void launch_gather_charges(hipStream_t st, int g, int m, int mpad64, const int* perm,
                           const double* xyz, const double* q, double Lx, double Ly, double4* cq,
                           double2* zr);
// fp32: FP32 tables and matrix cores, FP32 sums over 128 charges, FP64 beyond
void launch_b_sf_mfma(hipStream_t st, int g, int mpad, int nchunks, int nitems, const int4* items,
                      const int* sc_nx, const int* sc_ny, int ncolsort, int nxm, int nym, int nbz,
                      const double2* tab, const int* tile_nb, const int* toff, int pchunk,
                      double* part, int fp32, int sf16_nt);
void launch_b_sf_mfma_reduce(hipStream_t st, int ncolsort, int nchunks, int pchunk,
                             const int* tile_nb, const int* toff, const int* sc_lo,
                             const int* sc_len, const int* sc_koff, const int* n_index,
                             int n_total, const double* part, const double* w2, double* sfw);
void launch_b_sf_layer_reduce(hipStream_t st, int g, int ncolsort, int nchunks, int pchunk,
                              int nlayers, int nzt, int max_ncnt, const int* tile_nb,
                              const int* toff, const int* sc_lo, const int* sc_len,
                              const int* sc_koff, const int* n_index, const double* part,
                              const double* w2, const double2* pz, int M2, double* Tcat);
void launch_plane_phases(hipStream_t st, int nlayers, int nzt, const double* layer_fz,
                         double2* pz);
// planar electrodes: b from the projection parts (k_cg_tiles over the slot
// tiles), the real-space partials and the dipole term
void launch_b_final(hipStream_t st, int g, int n, int nslot, int nparts, const int* slot_of,
                    const double* Phi, const double* phir, int rchunks, const Buffers& b,
                    const double* dip, int dip_blocks, const double* cdip, double ke, void* out,
                    int out_is_f32);
int real_space_block_atoms();      // atom-map slots per workgroup of the real-space b kernel

int sf_table_rows(int nxm, int nym, int nbz);
int sf16_rows(int nxm, int nym, int nbz);      // float2 rows of the split-FP16 tables
void launch_b_sf_reduce(hipStream_t st, int nk, int mchunks, const double* part,
                        const double* w2, double* sfw);
void launch_b_kspace_project(hipStream_t st, int fp32, int n, int kchunks, const KCol* cols,
                             const int* chunk_col, const Buffers& b, const double* sfw,
                             double* part);
// planar electrodes: T(column, plane) then phi per atom over columns
void launch_b_layer_project(hipStream_t st, int n, int ncols, int nlayers, const KCol* cols,
                            const int* layer_of, const double* layer_fz, const Buffers& b,
                            const double* sfw, double2* T, double* part);
int layer_project_chunks(int ncols);
// factor-only inverse: X[r][j] = 1 for atom j < n of electrode r < n_e (rows
// x npad), and from Y = G^T A^-1 (rows a < n_e, stride ldy): u = A^-1 e,
// s = e^T u and the response S G (npad x n_e, row-major)
void launch_group_indicator(hipStream_t st, int n, int npad, int rows, const int* eid, int n_e,
                            double* X);
void launch_factor_response(hipStream_t st, int n, int npad, int n_e, const double* Y, int ldy,
                            double* u, double* s, double* sg);
void launch_pair_table(hipStream_t st, double alpha, double eta, double rc, double* tab);
void launch_b_real_space(hipStream_t st, int g, int n, int m, int mpad64, int rchunks,
                         const Buffers& b, int nmap, const double4* cq, const double2* zr,
                         double Lx, double Ly, double Lz, double rc, double* part, int wg_target,
                         const double* plane_tab);
// coefficients of g(r) as polynomials in r^2 on RP_N intervals of [0, rc]
// (RP_N x RP_REC doubles), for the planar real-space kernel
void pair_poly_table(double alpha, double eta, double rc, std::vector<double>& tab);
void launch_b_combine(hipStream_t st, int n, int kchunks, int rchunks, const double* phik,
                      const double* phir, const Buffers& b, const double* dip, int dip_blocks,
                      const double* cdip, double ke, void* out, int out_is_f32);

}  // namespace cpm
