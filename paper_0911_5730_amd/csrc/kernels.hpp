// Device data descriptors and host launchers of libbddc's kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace bddc {

constexpr int kNT = 256;   // threads per workgroup (4 wave64)

// Event pair that the next kernel launched from this host thread records
// around its own execution (set by the host timing facility, empty otherwise):
// the events are stamped at the start and end of the dispatch itself, so the
// interval excludes the launch gap before the kernel.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
inline thread_local LaunchEvents g_launch_events;

// A rejected launch (bad configuration, too much LDS) fails loudly.
void check_launch();

// Every launch of the library goes through here; arguments are converted to
// the kernel's parameter types before they are packed; a rejected launch
// throws.
template <class... P, class... A>
inline void launch_kernel(void (*k)(P...), dim3 grid, dim3 block, size_t shm, hipStream_t st, A... a) {
  const LaunchEvents ev = g_launch_events;
  g_launch_events = LaunchEvents{};
  hipExtLaunchKernelGGL(k, grid, block, static_cast<std::uint32_t>(shm), st, ev.start, ev.stop, 0u,
                        static_cast<P>(a)...);
  check_launch();
}

struct Khat16 {
  double v[16];   // 4x4 reference element matrix (k = 1), row-major, local node order CCW from (i,j)
};
// kernel modes of the operators without Dirichlet data: the constants, or
// the three rigid-body modes of plane elasticity (columns of the level's z)
constexpr int kMaxModes = 3;
// counters of the tail sums: per sum a top counter and kTailSlots slot
// counters, 16 words (64 bytes) apart
constexpr int kTailSlots = 64;
constexpr int kSlots = 256;   // slots of the slot sums: one per thread of a 256-thread workgroup
constexpr int kTailStride = 16 * (1 + kTailSlots);

struct Khat64 {
  double v[64];   // 8x8 elasticity element matrix (k = 1), row-major, dof 2 q + c of local node q
};

// Everything an apply kernel needs about one level, by value.
struct LevelDev {
  int nsub = 0;
  int nc = 0;                         // global coarse dofs of the level
  const int64_t* koff = nullptr;      // per substructure: offset of its dense matrix in K
  const int32_t* loc_ptr = nullptr;   // per substructure: start of its local dofs (size nsub+1)
  const int32_t* nint = nullptr;      // interior dofs
  const int32_t* nr = nullptr;        // interface non-corner dofs
  const int32_t* goff = nullptr;      // interface flat offset (size nsub+1)
  const int32_t* ioff = nullptr;      // interior flat offset (size nsub+1)
  const int32_t* coff = nullptr;      // local coarse flat offset (size nsub+1)
  const int32_t* int_gid = nullptr;   // interior flat -> level dof
  const int32_t* gam_gid = nullptr;   // interface flat -> level dof
  const int32_t* gam_iid = nullptr;   // interface flat -> interface index
  const int32_t* sh_ptr = nullptr;    // interface index -> sharers (flat interface entries)
  const int32_t* sh_flat = nullptr;
  const int32_t* cid = nullptr;       // local coarse flat -> global coarse id
  const double* K = nullptr;          // factored local matrices: L_II, L_GI, S (full)
  const double* delta = nullptr;      // stiffness-scaling weights, interface flat
  const double* T = nullptr;          // T_rr per substructure
  const int64_t* toff = nullptr;
  const double* Psi = nullptr;        // coarse basis on the interface, ng x ncs
  const int64_t* psioff = nullptr;
  double* y = nullptr;                // scratch: interior flat
  double* t = nullptr;                // scratch: interface flat
  double* a = nullptr;                // scratch: interface flat
  double* v = nullptr;                // scratch: interface flat
  double* b = nullptr;                // scratch: local coarse flat
  const int32_t* stop = nullptr;      // when non-null and *stop != 0 the apply kernels return at once
  const double* Linv = nullptr;       // levels >= 2: explicit inverse of L_II (lower, n_I x n_I)
  const int64_t* linvoff = nullptr;
  const int32_t* csh_ptr = nullptr;   // coarse dof -> local coarse flat entries (sharers)
  const int32_t* csh_flat = nullptr;
  // tiled elimination of large local matrices (64 x 64 tiles): per row tile
  // (interior tiles, then interface tiles) the first interior column tile that
  // holds a nonzero of the factor (the envelope; null = every tile), offsets
  // tproff; and the inverses of the interior diagonal tiles of L_II (64 x 64
  // column-major each), offsets woff
  const int32_t* tprof = nullptr;
  const int32_t* tproff = nullptr;
  // the same envelope per group of four rows (interior rows, then interface
  // rows, each from a group boundary): the first interior column any of the
  // four rows holds a nonzero in (entries left of it are zeros of the factor
  // and are not loaded), offsets rgfoff; null = column 0
  const int32_t* rgf = nullptr;
  const int32_t* rgfoff = nullptr;
  // large local matrices: the substructures in decreasing order of their
  // elimination work (workgroup b takes substructure order[b], so the largest
  // start first and the uneven sizes pack the CUs; null = in index order)
  const int32_t* order = nullptr;
  // level-1 sweeps: per substructure the end of the interior rows of each
  // panel's envelope (64-wide panels, then 32-wide), offsets srendoff; null =
  // every interior row below the panel
  const int32_t* srend = nullptr;
  const int32_t* srendoff = nullptr;
  const double* Wd = nullptr;
  const int64_t* woff = nullptr;
};

// All levels >= 2 and the coarsest solve in one workgroup (used when they are small).
constexpr int kMaxDeep = 6;
constexpr int kDeepNT = 1024;   // 16 wave64
struct DeepArgs {
  int nlev = 0;                       // number of deep levels (levels 2 .. L-1)
  LevelDev lv[kMaxDeep];
  double* rvec[kMaxDeep] = {};        // level vectors r_l (r_2 = level-1 coarse right-hand side)
  double* uvec[kMaxDeep] = {};        // u_l
  int nvec[kMaxDeep] = {};
  double* rc_last = nullptr;          // coarsest right-hand side and solution
  double* uc_last = nullptr;
  int ncL = 0;
  const double* LL = nullptr;         // coarsest Cholesky factor
  int n2 = 0;                         // r_2 gathered from the level-1 coarse sharers
  const int32_t* csh_ptr1 = nullptr;
  const int32_t* csh_flat1 = nullptr;
  const double* b1 = nullptr;
  const int32_t* stop = nullptr;
  int wstride = 0;                    // per-wave LDS scratch (doubles)
};

// One deep level (level 2) and the coarsest solve in one cooperative launch:
// one workgroup per level-2 substructure, its operators prefetched to LDS,
// three grid barriers between the phases that read other substructures' data.
constexpr int kCoopNT = 512;
constexpr int kCoopMeta = 9;   // per substructure: nI, ng, nr, ncs, n_sh, n_g1, goff, coff, n_phi
struct CoopDev {
  int nsub = 0;
  int ncL = 0;
  int nImax = 0, ngmax = 0, ncsmax = 0;
  int opmax = 0;                      // largest operator block (doubles)
  int idxmax = 0;                     // largest index block (ints)
  int cg_len = 0;                     // coarse gather block (ints)
  // per substructure: K_II^-1 | M^T (nI x ng) | T_rr | Psi | delta | phi weights
  const double* ops = nullptr;
  const double* Kinv = nullptr;       // setup only: K_II^-1 and M^T to pack (as in WideDev)
  const int64_t* kioff = nullptr;
  const double* Mt = nullptr;
  const int64_t* moff = nullptr;
  const int64_t* opoff = nullptr;
  // per substructure: int_gid | gam_gid | own | shp | shf | gp | gf | cid | phi_ptr | phi_ids
  const int32_t* idx = nullptr;
  const int64_t* idxoff = nullptr;
  const int32_t* meta = nullptr;      // kCoopMeta ints per substructure
  const int32_t* cg = nullptr;        // coarsest gather: ptr (ncL+1) | flat coarse indices
  const double* LLinv = nullptr;      // inverse of the coarsest Cholesky factor, ncL x ncL lower
  const double* b1 = nullptr;         // level-1 coarse contributions (input)
  double* t = nullptr;                // level-2 interface flat scratch
  double* b = nullptr;                // level-2 coarse flat scratch
  double* da = nullptr;               // level-2 interface flat scratch: delta T_rr g
  const int32_t* sub_of_flat = nullptr;   // level-2 interface flat entry -> substructure (setup only)
  double* u2 = nullptr;               // level-2 solution (output)
  const int32_t* stop = nullptr;
  unsigned* bar = nullptr;            // grid barrier: count, generation
  int* status = nullptr;
  // columns: b1 and u2 hold nrhs columns at strides ld_b1 and ld_u2, the
  // scratch t and da at ld_t, b at ld_b (every phase serves all columns)
  int nrhs = 1;
  int ld_b1 = 0, ld_u2 = 0, ld_t = 0, ld_b = 0;
};
size_t coop_lds(const CoopDev& C);
void launch_deep_coop(hipStream_t st, const CoopDev& C, bool cooperative);
void launch_coop_reset(hipStream_t st, const CoopDev& C);

// The fixed working array of the no-allocation solve: its device address on
// the current device, and a kernel that zeroes the first `bytes` of a buffer.
void* noalloc_scratch();
void launch_zero_bytes(hipStream_t st, void* p, size_t bytes);
void launch_pack_coop(hipStream_t st, const LevelDev& L, const CoopDev& C);
void launch_tri_inverse_dense(hipStream_t st, const double* L, int ld, int m, double* X);
int coop_max_blocks(size_t lds);

// One deep level with substructures too large for the cooperative kernel:
// row blocks of dense K_II^-1 and M^T = (K_GI K_II^-1)^T over many workgroups.
struct PcgScalars;
struct WideDev {
  LevelDev L;                         // level 2
  int nImax = 0, ngmax = 0;
  int rows1 = 8;                      // rows of [K_II^-1 ; M] per workgroup of the pre kernel
  int nchunk1 = 1, nchunk4 = 1;       // row chunks per substructure (pre, post)
  const double* Kinv = nullptr;       // n_I x n_I per substructure, column-major
  const int64_t* kioff = nullptr;
  const double* Mt = nullptr;         // M^T, n_I x n_G per substructure, column-major
  const int64_t* moff = nullptr;
  const double* b1 = nullptr;         // level-1 coarse contributions
  const int32_t* csh_ptr1 = nullptr;  // level-2 dof -> level-1 coarse flat entries
  const int32_t* csh_flat1 = nullptr;
  double* r2 = nullptr;               // level-2 right-hand side
  double* u2 = nullptr;               // level-2 solution
  int ncL = 0;
  const double* AL = nullptr;         // coarsest Cholesky factor, or A_L^-1 with coarse_inv
  int coarse_inv = 0;                 // the coarsest solve is a product with A_L^-1
  double* r3 = nullptr;               // with coarse_inv: coarsest right-hand sides and solutions,
  double* u3 = nullptr;               // nrhs columns at stride ld_3
  int ld_3 = 0;
  const int32_t* sub_of_flat = nullptr;   // level-2 interface flat entry -> substructure
  int nflat = 0;
  const int32_t* stop = nullptr;
  // columns: one grid slice per column c; b1, r2, u2 and the level-2 scratch
  // (L.y interior flat, L.t / L.a / L.v interface flat, L.b coarse flat)
  // hold nrhs columns at these strides
  int nrhs = 1;
  int cols1 = 1;                      // columns per workgroup of the pre kernel (set at its launch)
  int ld_b1 = 0, ld_r2 = 0, ld_u2 = 0, ld_i = 0, ld_g = 0, ld_c = 0;
  // several columns: r_2 is gathered once by a launch of its own, into r2
  // and (interior flat, stride ld_i) rIf, which the pre kernel reads
  double* rIf = nullptr;
  int gathered = 0;                   // (set at the pre kernel's launch)
  int n2 = 0, nflat_i = 0;            // level-2 dofs, interior flat entries
  // with sc: one more row of workgroups in the pre kernel, whose first sums the
  // level-1 r.r partials of each PCG column still iterating (rr_n partials at
  // stride rr_ld) into sc[c].rrs, in place of a launch of its own
  PcgScalars* sc = nullptr;
  const double* rr_part = nullptr;
  int rr_ld = 0, rr_n = 0;
};
void launch_wide_ops(hipStream_t st, const LevelDev& L, int nmax_ops, double* Kinv, const int64_t* kioff, double* Mt,
                     const int64_t* moff);
void launch_wide_pre(hipStream_t st, const WideDev& W);
// k_apply_restrict<true> for W.nrhs columns of W.r2 on W.L (the wide path's level-2 restriction)
void launch_wide_restrict(hipStream_t st, const WideDev& W, const int32_t* gam_map);
void launch_wide_coarse(hipStream_t st, const WideDev& W);
void launch_wide_post(hipStream_t st, const WideDev& W);

// state of the fused PCG iteration on the level-1 interface
struct PcgDev {
  struct PcgScalars* sc = nullptr;
  double *x = nullptr, *z = nullptr;
  double* r[2] = {nullptr, nullptr};         // residual, by iteration parity
  double* p[2] = {nullptr, nullptr};         // search direction, by iteration parity
  double* pq_part = nullptr;                 // per level-1 substructure: p_s^T S_s p_s
  double* rr_part = nullptr;                 // per level-1 substructure: owned r.r
  double* rz_part[2] = {nullptr, nullptr};   // per level-1 substructure, by iteration parity
  double* qloc = nullptr;                    // local Schur products, level-1 interface flat
  double* da = nullptr;                      // delta T_rr g, level-1 interface flat
  double* gflat = nullptr;                   // row-block path: g = delta r_k, level-1 interface flat
  const int32_t* phi_ptr = nullptr;          // per interface dof: its row of the delta-weighted
  const int32_t* phi_ids = nullptr;          //   coarse basis of all sharers (coarse ids, weights)
  const double* phi_w = nullptr;
  // per level-1 interface flat entry: the flat entries of all sharers of its
  // dof in sharer order, -1 past the last (null when a dof has more than four)
  const int4* shf4 = nullptr;
  int nif = 0;
  int nsub1 = 0;
  // wide interfaces: the product and the update/restriction take a workgroup
  // per 64-row block of each substructure (nrb blocks per substructure, 0:
  // one workgroup per substructure); the energies p_s^T S_s p_s are then left
  // per block, npq = nsub1 * max(1, nrb) partials per column
  int nrb = 0;
  int npq = 0;
  // full storage with each column starting on a 128-byte boundary (leading
  // dimension pad_ld(m, element bytes)), used with the row-block launches
  int fullpad = 0;
  int nblk = 1;                              // blocks of the interface average (rz partials)
  // 1: a one-block launch after each producing launch sums its partials once
  // into PcgScalars (rzs, pqs, rrs) and the consumers read that scalar; 2 (one
  // column): the producing launch's last block to finish does that sum
  // (counters tail_cnt, zeroed when a solve begins; several columns: as 1);
  // 3 (one column): slot sums (slotv) that every consuming block finishes;
  // 0: every consuming block sums the partials itself (cheaper when there are few)
  int fin = 0;
  unsigned int* tail_cnt = nullptr;          // counters of the three tail sums (3 kTailStride words)
  // finalize 3 (one column): slot t of a sum holds the partials of producing
  // blocks t, t + kSlots, ... summed in that order; values for p^T S p and r.z
  // by parity (3 kSlots doubles), one counter per slot and sum 64 bytes apart
  double* slotv = nullptr;
  unsigned int* slot_cnt = nullptr;          // 2 kSlots x 16 words
  // precision form of the interface preconditioner (bddc_precision): 0 FP64
  // T_rr and Psi; 1 FP32 copies of both; 2 T_rr in factored form
  //   T_rr = D^-1 W^T (I - Q Q^T) W D^-1,
  // D = diag(S_rr)^(1/2), W = inverse Cholesky factor of D^-1 S_rr D^-1 stored
  // as BF16 (packed lower triangle), Q an orthonormal basis of W D^-1 C_r^T in
  // FP32, D^-1 in FP32, Psi FP32.  Products of the reduced forms are formed in
  // FP64 (reduced storage, FP64 arithmetic); every vector stays FP64.
  int prec = 0;
  // 1: the product and update launches give the workgroups that the hardware
  // deals to one XCD (consecutive ids go round-robin over the eight) a
  // contiguous range of substructures, so neighbours share that XCD's L2
  int xcd = 0;
  const double* Sp = nullptr;       // S_s, packed lower triangle (column-major), offsets spoff
  int full = 0;                     // S_s and T_rr held as full column-major matrices instead (wide interfaces)
  const int64_t* spoff = nullptr;
  const double* Tp = nullptr;       // FP64 form: T_rr packed lower triangle, offsets tpoff
  const float* Tp32 = nullptr;      // FP32 form: T_rr packed lower triangle, offsets tpoff
  const int64_t* tpoff = nullptr;
  const uint16_t* W16 = nullptr;    // BF16 packed lower W, column-major (offsets toff)
  const float* Q32 = nullptr;       // FP32 Q, n_r x n_cr column-major (offsets croff)
  const float* Dinv = nullptr;      // D^-1 on the interface flat (first n_r entries of each substructure)
  const float* Psi32 = nullptr;     // FP32 Psi (offsets psioff)
  const int32_t* ncr = nullptr;     // constraint rows on the r dofs, per substructure
  const int64_t* croff = nullptr;
  // Blocked right-hand sides: column c of every PCG vector sits at c times
  // the stride of its kind, and sc[c] holds column c's scalars (sc[0] also
  // the chunk's iteration base and the all-columns-finished flag).  Each
  // launch reads an operator block once and applies it to every column still
  // iterating; a finished column's state is left as it was.
  int nrhs = 1;
  int ld_if = 0;       // interface vectors x, r, p, z
  int ld_flat = 0;     // interface flat: qloc, da
  int ld_cflat = 0;    // local coarse flat: b (level-1 coarse contributions)
  int ld_coarse = 0;   // level-1 coarse dofs: uc
  int ld_sub = 0;      // per-substructure partials: pq_part, rr_part
  int ld_blk = 0;      // per-block partials: rz_part
  double* b = nullptr;         // level-1 coarse contributions Psi^T g, per column
  const double* uc = nullptr;  // level-1 coarse correction, per column
};
constexpr int kMaxRhs = 8;   // columns of one blocked solve
// leading dimension of an m-row column-major matrix whose columns start on
// 128-byte boundaries
__host__ __device__ inline int pad_ld(int m, int elem_bytes) {
  const int e = 128 / elem_bytes;
  return (m + e - 1) / e * e;
}
constexpr int kCoarseInvMin = 512;   // coarse spaces at least this large are solved with A_L^-1

constexpr int kMaxHist = 4096;

struct PcgScalars {
  double rz, pq, alpha, beta, rr, bb, thr2, rtol2;
  double rzs[2], pqs, rrs;   // summed partials of the fused iteration (r.z by parity, p^T S p, r.r)
  int32_t it_base;           // PCG iteration of offset 0 in the launches of the current chunk
  int32_t pad2;
  int32_t iters, maxit, done;
  int32_t all_done;          // column 0 only: every column of the blocked solve has finished
  double alphas[kMaxHist];
  double betas[kMaxHist];
};

// setup
void launch_assemble_l1(hipStream_t st, int nsub, const int64_t* koff, const int32_t* loc_ptr,
                        const int32_t* nint, const int32_t* node_el, const int32_t* sub_el_ptr,
                        const int32_t* el_gid, const int32_t* el_loc, const double* coeff,
                        const Khat16& khat, double* K, double* diagK, const int32_t* goff, int* status);
// the same for plane elasticity: eight element dofs (node_el codes with three position bits)
void launch_assemble_l1_elastic(hipStream_t st, int nsub, const int64_t* koff, const int32_t* loc_ptr,
                                const int32_t* nint, const int32_t* node_el, const int32_t* sub_el_ptr,
                                const int32_t* el_gid, const int32_t* el_loc, const double* coeff,
                                const Khat64& khat, double* K, double* diagK, const int32_t* goff, int* status);
void launch_assemble_coarse(hipStream_t st, int nsub, const int64_t* koff, const int32_t* loc_ptr,
                            const int32_t* nint, const int32_t* child_ptr, const int32_t* child_id,
                            const int32_t* child_map_off, const int32_t* child_map, const double* Ac,
                            const int64_t* acoff, const int32_t* nc_child, double* K, double* diagK,
                            const int32_t* goff);
void launch_weights(hipStream_t st, int nflat, const int32_t* flat_iid, const int32_t* sh_ptr,
                    const int32_t* sh_flat, const double* diagK, double* delta);
// PCG product and update/restriction by 64-row blocks (k_pcg_rows.hip)
size_t pcg_rows_lds(int ngmax, int nrhs);
int pcg_rows_blocks(int ngmax);
void launch_pcg_matvec_rows(hipStream_t st, const LevelDev& L, int ngmax, const PcgDev& P, int u);
void launch_pcg_update_rows(hipStream_t st, const LevelDev& L, const PcgDev& P, int u);
void launch_pcg_restrict_rows(hipStream_t st, const LevelDev& L, int ngmax, const PcgDev& P, int u);
// local matrices of any size: left-looking blocked elimination with 64 x 64
// tiles staged in LDS and FP64 MFMA products (k_bigchol.hip)
void launch_partial_chol_big(hipStream_t st, const LevelDev& L, double* K, double* Wd, int* status);
// interior solves of many columns with the tiled factor (k_tile.hip):
//   pre:     y = L_II^-1 r_I, t = L_GI y  (condensation / interior pre-correction)
//   recover: u_G = x, u_I = L_II^-T (y - L_GI^T x)  (y is overwritten by u_I)
void launch_tile_pre_cols(hipStream_t st, const LevelDev& L, const double* r, int64_t ldr, double* y, int ldy,
                          double* t, int ldt, int R);
void launch_tile_recover_cols(hipStream_t st, const LevelDev& L, const double* x, int ldx, double* y, int ldy,
                              double* u, int64_t ldu, int R, int ngmax);
size_t partial_chol_big_lds();
void launch_partial_chol(hipStream_t st, int nsub, int nmax, const int64_t* koff, const int32_t* loc_ptr,
                         const int32_t* nint, double* K, int* status);
size_t partial_chol_lds(int nmax);
int partial_chol_mfma_nb(int nmax);
bool sweep_fits(int nmax);
void launch_sweep_pre(hipStream_t st, const LevelDev& L, const double* r);
void launch_sweep_post(hipStream_t st, const LevelDev& L, double* u, const int32_t* gam_map);
void launch_sweep_recover(hipStream_t st, const LevelDev& L, const double* x, double* u);
// condensation (y = L_II^-1 r_I, t = L_GI y) and interior recovery for R <= kMaxRhs
// columns at once (column c of each vector at c times its stride)
void launch_sweep_pre_cols(hipStream_t st, const LevelDev& L, const double* r, int64_t ldr, double* y, int ldy, double* t,
                           int ldt, int R);
void launch_sweep_recover_cols(hipStream_t st, const LevelDev& L, const double* x, int ldx, const double* y, int ldy,
                               double* u, int64_t ldu, int R);
size_t constrained_factor_lds(int ng, int n_r, int n_cr, int ncs);
void launch_constrained_factor_lds(hipStream_t st, int nsub, size_t lds, const int64_t* koff, const int32_t* loc_ptr,
                                   const int32_t* nint, const int32_t* nr, const int32_t* ncr, const int64_t* croff,
                                   const double* Cr, const double* K, double* T, const int64_t* toff, double* Psi,
                                   const int64_t* psioff, double* Ac, const int64_t* acoff, int* status);
size_t tri_inverse_lds(int nImax);
void launch_tri_inverse_lds(hipStream_t st, int nsub, int nImax, const int64_t* koff, const int32_t* loc_ptr,
                            const int32_t* nint, const double* K, double* Linv, const int64_t* linvoff);
size_t partial_chol_mfma_lds(int nmax);
void launch_partial_chol_mfma(hipStream_t st, int nsub, int nmax, const int64_t* koff, const int32_t* loc_ptr,
                              const int32_t* nint, double* K, int* status);
void launch_build_cr(hipStream_t st, int nsub, const int32_t* sub_inc_ptr, const int32_t* sub_inc,
                     const int32_t* inc_edge, const int32_t* inc_fptr, const int32_t* inc_fpos,
                     const int32_t* edge_nsc, const int32_t* edge_ne, const int32_t* edge_m,
                     const int64_t* qoff, const double* Q, const int32_t* nr, const int32_t* ncr,
                     const int64_t* croff, double* Cr);
void launch_coarse_z(hipStream_t st, int nc, const int32_t* cd_dof, const int32_t* cd_col,
                     const int32_t* edge_ptr, const int32_t* edge_dof, const int64_t* qoff,
                     const double* Q, const double* z, int nz, int zld, double* znext);
void launch_constrained_factor(hipStream_t st, int nsub, const int64_t* koff, const int32_t* loc_ptr,
                               const int32_t* nint, const int32_t* nr, const int32_t* ncr,
                               const int64_t* croff, const double* Cr, const double* K, double* T,
                               const int64_t* toff, double* Psi, const int64_t* psioff, double* Ac,
                               const int64_t* acoff, double* work, const int64_t* woff, int* status);
void launch_coarsest_factor(hipStream_t st, int nsub, int nc, const int32_t* cptr, const int32_t* cid,
                            const double* Ac, const int64_t* acoff, double* AL, int* status);
// the assembly of launch_coarsest_factor without the factorization (AL zeroed first)
void launch_coarsest_assemble(hipStream_t st, int nsub, int nc, const int32_t* cptr, const int32_t* cid,
                              const double* Ac, const int64_t* acoff, double* AL);

// adaptive
void launch_pair_schur(hipStream_t st, int ninc, int ngmax, const int32_t* inc_sub, const int32_t* inc_fptr,
                       const int32_t* inc_fpos, const int64_t* koff, const int32_t* loc_ptr,
                       const int32_t* nint, const double* K, const int64_t* inc_off, double* Shat,
                       double* Sff, int* status, double* ws = nullptr, const int64_t* wsoff = nullptr);
// LDS bytes of one pair Schur complement (interface of ngmax dofs) and one
// pair eigenproblem; with a global workspace each block takes the same
// number of bytes from it instead
size_t pair_schur_lds(int ngmax);
size_t pair_eig_lds(int nemax, int nvmax);
void launch_pair_eig(hipStream_t st, int nedge, int nemax, int nvmax, const int32_t* edge_s, const int32_t* edge_t,
                     const int32_t* edge_nsc, const int32_t* edge_ne, const int32_t* edge_fdof,
                     const int32_t* edge_fptr, const int32_t* inc_fptr, const int32_t* inc_fpos,
                     const int32_t* goff, const double* diagK, const uint8_t* floating, const double* z, int nz,
                     int zld,
                     const double* Shat, const double* Sff, const int64_t* inc_off, double tau, double* lam,
                     const int64_t* lamoff, double* Q, const int64_t* qoff, int32_t* nsel, int32_t* nkept,
                     int* status, double* ws = nullptr, const int64_t* wsoff = nullptr);

// apply and PCG
void launch_apply_pre(hipStream_t st, const LevelDev& L, int nImax, int ngmax, const double* r);
void launch_apply_restrict(hipStream_t st, const LevelDev& L, int ngmax, const double* r,
                           const int32_t* gam_map, int use_t);
void launch_coarse_gather(hipStream_t st, int nc, const int32_t* csh_ptr, const int32_t* csh_flat,
                          const double* b, double* rc, const int32_t* stop);
// large coarsest problems: A_L^-1 in place of A_L (block Gauss-Jordan; P is
// 64 x 64 and T n x 64 scratch), and the solve as a product with it
void launch_coarsest_inverse(hipStream_t st, int n, double* A, double* P, double* T, int* status);
void launch_coarse_gather_cols(hipStream_t st, int nc, const int32_t* csh_ptr, const int32_t* csh_flat,
                               const double* b, int64_t ldb, double* r, int64_t ldr, int ncols, const int32_t* stop);
void launch_coarse_inv_apply(hipStream_t st, int n, const double* Ainv, const double* r, int64_t ldr, double* u,
                             int64_t ldu, int ncols, const int32_t* stop);
// k_apply_pre / k_recover for R <= kMaxRhs columns (LDS apply_cols_lds(R, nImax, ngmax))
size_t apply_cols_lds(int R, int nImax, int ngmax);
void launch_apply_pre_cols(hipStream_t st, const LevelDev& L, int nImax, int ngmax, const double* r, int64_t ldr,
                           double* y, int ldy, double* t, int ldt, int R);
void launch_recover_cols(hipStream_t st, const LevelDev& L, int nImax, int ngmax, const double* x, int ldx,
                         const double* y, int ldy, double* u, int64_t ldu, int R);
void launch_coarsest_solve(hipStream_t st, int nc, const double* Lc, const double* rc, double* uc,
                           const int32_t* stop);
void launch_coarse_direct_cols(hipStream_t st, int nc, const int32_t* csh_ptr, const int32_t* csh_flat,
                               const double* b, int ldb, const double* Lc, double* uc, int ldu, int ncols,
                               const int32_t* stop);
void launch_apply_prolong(hipStream_t st, const LevelDev& L, int ncsmax, const double* uc);
void launch_apply_post(hipStream_t st, const LevelDev& L, int nImax, int ngmax, double* u,
                       const int32_t* gam_map, int interior);
void launch_schur_local(hipStream_t st, const LevelDev& L, int ngmax, const double* p, double* qloc);
void launch_gather_dot(hipStream_t st, int nblk, int nif, const int32_t* sh_ptr, const int32_t* sh_flat,
                       const double* qloc, const double* p, double* q, double* partial);
void launch_dot_partial(hipStream_t st, int nblk, int n, const double* a, const double* b, double* partial);
void launch_scalar(hipStream_t st, int which, int nblk, const double* partial, PcgScalars* sc);
void launch_update_xr(hipStream_t st, int nblk, int n, const PcgScalars* sc, const double* p, const double* q,
                      double* x, double* r, double* partial);
void launch_update_p(hipStream_t st, int nblk, int n, const PcgScalars* sc, const double* z, double* p, int first);
void launch_condense(hipStream_t st, int nif, const int32_t* sh_ptr, const int32_t* sh_flat,
                     const int32_t* iface_gid, const double* f, const double* t, double* r, double* x);
void launch_recover(hipStream_t st, const LevelDev& L, int nImax, int ngmax, const double* x, double* u);
void launch_copy(hipStream_t st, int n, const double* a, double* b);

// levels >= 2: explicit inverse of the interior factor; fused deep apply
void launch_tri_inverse(hipStream_t st, int nsub, int nImax, const int64_t* koff, const int32_t* loc_ptr,
                        const int32_t* nint, const double* K, double* Linv, const int64_t* linvoff);
size_t deep_lds(int wstride, int ncL);
void launch_deep(hipStream_t st, const DeepArgs& A);
void launch_apply_pre_inv(hipStream_t st, const LevelDev& L, int nImax, int ngmax, const double* r);
void launch_apply_post_inv(hipStream_t st, const LevelDev& L, int nImax, int ngmax, double* u);

// fused PCG iteration kernels (level-1 interface)
void launch_pcg_matvec(hipStream_t st, const LevelDev& L, int ngmax, const PcgDev& P, int u);
// which: 0 p^T S p (-> pqs), 1 r.r (-> rrs), 2 r.z of iteration it (-> rzs[it & 1]);
// iteration numbers are it = sc->it_base + u, or 0 for u < 0
void launch_pcg_sum(hipStream_t st, const PcgDev& P, int which, int u);
void launch_tail_reset(hipStream_t st, const PcgDev& P);
void launch_slot_reset(hipStream_t st, const PcgDev& P);
void launch_pcg_advance(hipStream_t st, const PcgDev& P, int n);
void launch_round_factors(hipStream_t st, const LevelDev& L, const PcgDev& P, int nrmax, int ncrmax, const double* Cr,
                          int* status);
void launch_pack_pcg(hipStream_t st, const LevelDev& L, const PcgDev& P);
void launch_pcg_update_restrict(hipStream_t st, const LevelDev& L, int ngmax, int nrmax, int ncsmax, const PcgDev& P,
                                int u);
void launch_pcg_prolong_post(hipStream_t st, const LevelDev& L, const PcgDev& P, int u);
void launch_build_phi(hipStream_t st, const LevelDev& L, int nif, const int32_t* sub_of_flat, const int32_t* phi_ptr,
                      int32_t* phi_ids, double* phi_w, const float* psi32);

}  // namespace bddc
