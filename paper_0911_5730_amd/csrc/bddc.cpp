// libbddc: host orchestration of adaptive-multilevel BDDC on one GPU.
//
// bddc_setup follows the adaptive setup algorithm of Section 5 level by level:
// topology and coarse-dof candidates (host, integer), then on the device the
// local matrices, stiffness-scaling weights, interior elimination, per-edge
// eigenproblems, constrained local factors with the energy-minimal coarse
// basis and the next level's matrices; the last level is factored directly.
// bddc_apply runs Algorithm "Multilevel BDDC"; bddc_solve runs PCG on the
// level-1 interface (Section 5, reduction of level 1 to the interfaces).
#include <atomic>
#include <climits>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <unordered_map>

#include "common.hpp"
#include "kernels.hpp"
#include "topology.hpp"

namespace bddc {

// handles alive in the process; the cooperative deep kernel uses the
// cooperative launch API whenever another handle may be running beside it
std::atomic<int> g_live_handles{0};

void check_launch() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) fail(BDDC_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}

namespace {
std::mutex g_pinned_mu;
std::vector<std::pair<void*, size_t>> g_pinned_free;   // buffers not in use
std::map<void*, size_t> g_pinned_size;                 // every buffer ever made
}  // namespace

void* pinned_acquire(size_t bytes) {
  std::lock_guard<std::mutex> lk(g_pinned_mu);
  size_t best = g_pinned_free.size();
  for (size_t i = 0; i < g_pinned_free.size(); ++i)
    if (g_pinned_free[i].second >= bytes && (best == g_pinned_free.size() || g_pinned_free[i].second < g_pinned_free[best].second))
      best = i;
  if (best < g_pinned_free.size()) {
    void* p = g_pinned_free[best].first;
    g_pinned_free.erase(g_pinned_free.begin() + best);
    return p;
  }
  size_t n = 1 << 20;
  while (n < bytes) n <<= 1;
  void* p = nullptr;
  BDDC_HIP(hipHostMalloc(&p, n, hipHostMallocDefault));
  g_pinned_size[p] = n;
  return p;
}

void pinned_release(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pinned_mu);
  auto it = g_pinned_size.find(p);
  if (it != g_pinned_size.end()) g_pinned_free.push_back({p, it->second});
}

Staging::~Staging() {
  if (!buf_) return;
  if (deferred_) {
    deferred_->push_back(buf_);
    return;
  }
  (void)hipStreamSynchronize(st_);
  pinned_release(buf_);
}

void Staging::flush() {
  if (items_.empty()) return;
  std::sort(items_.begin(), items_.end(), [](const Item& a, const Item& b) { return a.dst < b.dst; });
  // runs of destinations separated by alignment padding only
  std::vector<std::pair<size_t, size_t>> runs;   // [first item, last item]
  size_t total = 0;
  for (size_t i = 0; i < items_.size(); ++i) {
    if (i > 0 && items_[i].dst >= items_[i - 1].dst + items_[i - 1].bytes &&
        items_[i].dst - (items_[i - 1].dst + items_[i - 1].bytes) < 256)
      runs.back().second = i;
    else
      runs.push_back({i, i});
  }
  for (auto& r : runs) total += (size_t)(items_[r.second].dst + items_[r.second].bytes - items_[r.first].dst);
  if (buf_) {
    if (deferred_) {
      deferred_->push_back(buf_);
    } else {
      (void)hipStreamSynchronize(st_);
      pinned_release(buf_);
    }
  }
  buf_ = pinned_acquire(total);
  char* host = static_cast<char*>(buf_);
  size_t off = 0;
  for (auto& r : runs) {
    char* d0 = items_[r.first].dst;
    const size_t len = (size_t)(items_[r.second].dst + items_[r.second].bytes - d0);
    for (size_t i = r.first; i <= r.second; ++i) std::memcpy(host + off + (items_[i].dst - d0), items_[i].src, items_[i].bytes);
    BDDC_HIP(hipMemcpyAsync(d0, host + off, len, hipMemcpyHostToDevice, st_));
    off += len;
  }
  items_.clear();
}

namespace {
struct DevBlock {
  int dev;
  size_t size;
};
std::mutex g_dev_mu;
std::multimap<size_t, std::pair<int, void*>> g_dev_free;   // size -> (device, pointer)
std::map<void*, DevBlock> g_dev_blocks;                     // every block made
}  // namespace

void* device_acquire(size_t bytes) {
  int dev = 0;
  BDDC_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    for (auto it = g_dev_free.lower_bound(bytes); it != g_dev_free.end() && it->first <= 2 * bytes + (1 << 20); ++it) {
      if (it->second.first != dev) continue;
      void* p = it->second.second;
      g_dev_free.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  const size_t n = (bytes + 4095) & ~size_t(4095);
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    // give the cached blocks back and try once more
    {
      std::lock_guard<std::mutex> lk(g_dev_mu);
      for (auto it = g_dev_free.begin(); it != g_dev_free.end();) {
        if (it->second.first == dev) {
          (void)hipFree(it->second.second);
          g_dev_blocks.erase(it->second.second);
          it = g_dev_free.erase(it);
        } else {
          ++it;
        }
      }
    }
    (void)hipGetLastError();
    e = hipMalloc(&p, n);
    if (e != hipSuccess)
      fail(e == hipErrorOutOfMemory ? BDDC_ENOMEM : BDDC_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(g_dev_mu);
  g_dev_blocks[p] = DevBlock{dev, n};
  return p;
}

void device_release(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_dev_blocks.find(p);
  if (it != g_dev_blocks.end()) g_dev_free.insert({it->second.size, {it->second.dev, p}});
}

// ---------------------------------------------------------------------------
// Kernel timing for measurement tools: while armed for one kernel name, every
// launch of that kernel is bracketed by HIP events on its own stream, with the
// launch's algorithmic bytes and flops recorded beside it.
namespace timing {
struct Rec {
  hipEvent_t a, b;
  double bytes, flops;
  int tag;   // PCG iteration of the launch (-1 outside PCG)
};
std::mutex mu;
std::string target;
std::vector<Rec> recs;
std::vector<hipEvent_t> pool;
thread_local int current_tag = -1;   // set by the PCG driver while it enqueues an iteration
int every = 1;            // time one in `every` launches of the target
int64_t seen = 0;         // launches of the target since timing_start

size_t mark() {
  std::lock_guard<std::mutex> lk(mu);
  return recs.size();
}

bool active() {
  std::lock_guard<std::mutex> lk(mu);
  return !target.empty();
}

// drop the records from `from` on whose tag is >= limit: launches enqueued
// after convergence return at once and move no data
void prune(size_t from, int limit) {
  std::lock_guard<std::mutex> lk(mu);
  if (from >= recs.size()) return;
  std::vector<Rec> keep(recs.begin(), recs.begin() + from);
  for (size_t i = from; i < recs.size(); ++i) {
    if (recs[i].tag >= limit) {
      pool.push_back(recs[i].a);
      pool.push_back(recs[i].b);
    } else {
      keep.push_back(recs[i]);
    }
  }
  recs.swap(keep);
}

hipEvent_t get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  BDDC_HIP(hipEventCreate(&e));
  return e;
}

class Scope {
 public:
  Scope(const char* name, double bytes, double flops, int tag_shift = 0) {
    std::lock_guard<std::mutex> lk(mu);
    if (target.empty() || target != name) return;
    if (seen++ % every != 0) return;
    rec_.a = get_event();
    rec_.b = get_event();
    rec_.bytes = bytes;
    rec_.flops = flops;
    rec_.tag = current_tag < 0 ? -1 : current_tag + tag_shift;
    g_launch_events = LaunchEvents{rec_.a, rec_.b};   // taken by the scope's first launch
    on_ = true;
  }
  ~Scope() {
    if (!on_) return;
    std::lock_guard<std::mutex> lk(mu);
    if (g_launch_events.start == rec_.a) {   // nothing was launched
      g_launch_events = LaunchEvents{};
      pool.push_back(rec_.a);
      pool.push_back(rec_.b);
      return;
    }
    recs.push_back(rec_);
  }

 private:
  bool on_ = false;
  Rec rec_{};
};
}  // namespace timing

// host wall-clock breakdown printed to stderr when BDDC_HOST_TIMING is set
class HostClock {
 public:
  HostClock() : on_(getenv("BDDC_HOST_TIMING") != nullptr), t_(std::chrono::steady_clock::now()) {}
  void lap(const char* what) {
    if (!on_) return;
    const auto now = std::chrono::steady_clock::now();
    fprintf(stderr, "libbddc host %-18s %8.3f ms\n", what, std::chrono::duration<double, std::milli>(now - t_).count());
    t_ = now;
  }

 private:
  bool on_;
  std::chrono::steady_clock::time_point t_;
};

namespace {

constexpr size_t kLdsLimit = 64 * 1024 - 1024;   // dynamic LDS of the kernels sized for several blocks per CU
constexpr size_t kLdsMax = 160 * 1024;          // LDS of one CU, all of it usable by one block on gfx950

// Interior elimination: 64-wide LDS panels with an MFMA trailing update, unless
// the substructure is too large for a 16-wide panel in LDS or BDDC_CHOL_PATH=lds16
// (16-wide panels on the vector units) or =big.
bool use_mfma_chol(int nmax) {
  const char* env = getenv("BDDC_CHOL_PATH");
  if (env && (std::string(env) == "lds16" || std::string(env) == "big")) return false;
  return partial_chol_mfma_nb(nmax) >= 16 && partial_chol_mfma_lds(nmax) <= kLdsMax;
}

// Local matrices too large for the panel kernels (or BDDC_CHOL_PATH=big): the
// left-looking tiled elimination, whose LDS does not depend on the size.
bool use_big_chol(int nmax) {
  const char* env = getenv("BDDC_CHOL_PATH");
  if (env && std::string(env) == "big") return true;
  if (env && std::string(env) == "lds16") return false;
  return !use_mfma_chol(nmax);
}

// Level 1: the interior elimination by the tiled kernel at any size, for the
// tiled block substitutions of the interface-reduced solve (its condensation
// and recovery; the set-up also leaves the tiles' envelope and diagonal
// inverses), unless BDDC_IR_PATH=sweep or another elimination path is forced.
// Deeper levels: the tiled kernel only where the panels do not fit.
bool level_big_chol(int ell, int nmax) {
  if (use_big_chol(nmax)) return true;
  if (ell != 1) return false;
  const char* env = getenv("BDDC_CHOL_PATH");
  if (env && *env) return false;
  const char* ir = getenv("BDDC_IR_PATH");
  return !(ir && std::string(ir) == "sweep");
}

// Level-1 interior sweeps streamed through LDS panels unless the substructures
// are too large for them or BDDC_SWEEP=off.
bool use_sweep(int nmax) {
  const char* env = getenv("BDDC_SWEEP");
  if (env && std::string(env) == "off") return false;
  return sweep_fits(nmax);
}

// Local coarse-space factorization and interior triangular inverse in LDS,
// unless the substructure does not fit or BDDC_SETUP_PATH=global.
bool use_lds_setup() {
  const char* env = getenv("BDDC_SETUP_PATH");
  return !(env && std::string(env) == "global");
}

inline uint64_t pkey(int s, int t) {
  return (static_cast<uint64_t>(static_cast<uint32_t>(s)) << 32) | static_cast<uint32_t>(t);
}

template <class T>
std::vector<T> prefix(const std::vector<T>& cnt) {
  std::vector<T> p(cnt.size() + 1, 0);
  for (size_t i = 0; i < cnt.size(); ++i) p[i + 1] = p[i] + cnt[i];
  return p;
}

int dofs_per_node(int element) { return element == BDDC_Q1_ELASTIC ? 2 : 1; }

// Plane-strain elasticity (Section 6: lambda = 1, mu = 2) on an hx x hy
// rectangle, bilinear displacements: K = int B^T D B with strains (e_xx,
// e_yy, g_xy) and D the plane-strain stiffness, by the tensor 2-point Gauss
// rule (exact for these integrands).  Dof 2 q + c is component c of local
// node q (CCW from (i,j)); row-major 8 x 8.
Khat64 elastic_element_matrix(int nx, int ny) {
  const double lam = 1.0, mu = 2.0;
  const double hx = 1.0 / nx, hy = 1.0 / ny;
  const double Dm[3][3] = {{lam + 2 * mu, lam, 0.0}, {lam, lam + 2 * mu, 0.0}, {0.0, 0.0, mu}};
  const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  const double xq[4] = {0, 1, 1, 0}, yq[4] = {0, 0, 1, 1};   // local node positions on the unit square
  Khat64 k{};
  for (double xi : gp)
    for (double eta : gp) {
      double B[3][8] = {};
      for (int q = 0; q < 4; ++q) {
        // bilinear shape function of node q: (xq ? xi : 1 - xi) (yq ? eta : 1 - eta)
        const double fx = xq[q] ? xi : 1.0 - xi, fy = yq[q] ? eta : 1.0 - eta;
        const double dx = (xq[q] ? 1.0 : -1.0) * fy / hx;   // d/dx
        const double dy = (yq[q] ? 1.0 : -1.0) * fx / hy;   // d/dy
        B[0][2 * q] = dx;
        B[1][2 * q + 1] = dy;
        B[2][2 * q] = dy;
        B[2][2 * q + 1] = dx;
      }
      const double w = 0.25 * hx * hy;
      for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
          double acc = 0.0;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) acc += B[i][a] * Dm[i][j] * B[j][b];
          k.v[a * 8 + b] += w * acc;
        }
    }
  return k;
}

// reference element matrices (k = 1) of an hx x hy rectangle, local nodes
// (i,j), (i+1,j), (i+1,j+1), (i,j+1)
Khat16 element_matrix(int element, int nx, int ny) {
  const double rho = (1.0 / ny) / (1.0 / nx);   // hy / hx
  Khat16 k{};
  if (element == BDDC_Q1) {
    // (hy/hx) * int dphi/dx dphi/dx + (hx/hy) * int dphi/dy dphi/dy on the unit square
    const double ax[16] = {2, -2, -1, 1, -2, 2, 1, -1, -1, 1, 2, -2, 1, -1, -2, 2};
    const double ay[16] = {2, 1, -1, -2, 1, 2, -2, -1, -1, -2, 2, 1, -2, -1, 1, 2};
    for (int i = 0; i < 16; ++i) k.v[i] = (rho * ax[i] + ay[i] / rho) / 6.0;
  } else {
    // two P1 triangles split along the SW-NE diagonal
    const double a = rho, b = 1.0 / rho;
    const double m[16] = {a + b, -a, 0, -b, -a, a + b, -b, 0, 0, -b, a + b, -a, -b, 0, -a, a + b};
    for (int i = 0; i < 16; ++i) k.v[i] = 0.5 * m[i];
  }
  return k;
}

}  // namespace

// ---------------------------------------------------------------------------
// slots per edge for the components of its averages: -1 (mixed), 0, 1
constexpr int kMaxComp = 3;

struct Level {
  int ell = 1;
  Topology topo;
  int nsub = 0, n = 0;
  // displacement component of each dof (0 for scalar problems, -1 for a coarse
  // dof that mixes components), of each coarse dof, and of each edge average
  // (kMaxComp slots per edge)
  std::vector<int8_t> comp, cd_comp, edge_ccomp;
  // layout
  std::vector<int64_t> koff;
  std::vector<int32_t> goff, ioff, coff;
  int nflat_g = 0, nflat_i = 0, nflat_c = 0;
  std::vector<int32_t> int_gid, gam_gid, gam_iid, iface_dof, sh_ptr, sh_flat;
  std::vector<int32_t> nr_v;
  int nImax = 0, ngmax = 0, nmax = 0, ncsmax = 0, nrmax = 0;
  // edges and (substructure, edge) incidences
  int nedge = 0;
  std::vector<int32_t> edge_nsc, edge_ne, edge_fptr, edge_fdof;
  std::vector<int32_t> inc_sub, inc_edge, inc_fptr, inc_fpos;
  std::vector<int32_t> sub_inc_ptr, sub_inc;
  std::vector<int64_t> inc_off, lamoff, qoff;
  int nemax = 0, nvmax = 0;
  // pair Schur complements / pair eigenproblems too large for LDS work in a
  // global workspace: per incidence / per edge offsets (doubles), empty if not
  std::vector<int64_t> schws_off, eigws_off;
  // coarse dofs
  std::vector<int32_t> edge_m, edge_nsel;
  std::vector<double> lam;
  int nc = 0;
  std::vector<int32_t> cid, csh_ptr, csh_flat, cd_dof, cd_col, ncr;
  std::vector<int64_t> croff, toff, psioff, acoff, cwoff;
  double omega = 0.0;
  int n_adaptive = 0;
  std::vector<int32_t> agglom_of;   // level-(l+1) substructure of each substructure
  // algorithmic bytes / flops of one launch of each kernel at this level
  double by_schur = 0, by_restrict_ir = 0, by_restrict_fs = 0, by_update_restrict = 0, by_prolong = 0, by_post_ir = 0,
         by_post_fs = 0, by_pre = 0, fl_chol = 0, by_chol = 0;
  // device
  Arena arena_a, arena_b, arena_pcg;
  struct {
    int32_t *loc_ptr, *nint, *nr, *goff, *ioff, *int_gid, *gam_gid, *gam_iid, *iface_dof, *sh_ptr, *sh_flat;
    int64_t* koff;
    double *K, *diagK, *delta;
    // level-1 assembly
    int32_t *node_el, *sub_el_ptr, *el_gid, *el_loc;
    double* coeff;
    // level >= 2 assembly
    int32_t *child_ptr, *child_id, *child_map_off, *child_map;
    // incidences / edges
    int32_t *inc_sub, *inc_edge, *inc_fptr, *inc_fpos, *sub_inc_ptr, *sub_inc;
    int32_t *edge_s, *edge_t, *edge_nsc, *edge_ne, *edge_fdof, *edge_fptr, *edge_ptr, *edge_dof;
    uint8_t* floating;
    int64_t *inc_off, *lamoff, *qoff, *schws_off, *eigws_off;
    double *Shat, *Sff, *lam, *Q, *schws, *eigws;
    int32_t *nsel, *nkept;
    double* z;
    // coarse
    int32_t *edge_m, *coff, *cid, *csh_ptr, *csh_flat, *cd_dof, *cd_col, *ncr, *ncs;
    int64_t *croff, *toff, *psioff, *acoff, *cwoff;
    double *Cr, *T, *Psi, *Ac, *cwork, *znext;
    // scratch
    double *y, *t, *a, *v, *b, *rc, *uc, *qloc;
    double* Linv;
    int64_t* linvoff;
    // tiled elimination (large local matrices): envelope per row tile, inverses of the diagonal tiles
    int32_t *tprof, *tproff, *rgf, *rgfoff;
    double* Wd;
    int64_t* woff;
    // level-1 sweeps: the envelope's interior row ends per panel
    int32_t *srend, *srendoff;
    // large local matrices: workgroup -> substructure, largest first
    int32_t* order;
  } d{};
  bool sweep_env = false;
  bool has_order = false;
  bool has_rgf = false;
  std::vector<int64_t> linvoff;
  bool big = false;   // interior elimination by the tiled kernel
  LevelDev dev;
};

// A PCG solve in progress on a handle: its load, columns, iteration count
// and the interior-solve form chosen at its start.
struct PcgRun {
  bool active = false;
  bool stepwise = false;          // begun by bddc_solve_begin
  hipStream_t saved_stream = nullptr;
  const double* f = nullptr;
  int64_t ld = 0;
  int R = 0, maxit = 0, it = 0;
  bool sweep = false, tiles = false, blocked = false;
  size_t tmark = 0;
};

}  // namespace bddc

struct bddc_ctx {
  int nx = 0, ny = 0, L = 2, element = 0, constraints = 0, precision = 0;
  int nz = 1;   // kernel modes of the operators without Dirichlet data (elasticity: 3 rigid-body modes)
  double tau = 0;
  int64_t n_free = 0;
  hipStream_t stream = nullptr;
  std::vector<std::unique_ptr<bddc::Level>> levels;
  bddc::Arena top;        // coarsest factor, PCG state, status flag
  double* AL = nullptr;
  int ncL = 0;
  // coarse spaces of kCoarseInvMin dofs and more: AL holds A_L^-1 (block
  // Gauss-Jordan at set-up) and every coarsest solve is a product with it;
  // P / T are the sweep's scratch, coarse_r / coarse_u kMaxRhs columns of
  // coarsest right-hand sides and solutions at stride ld_cr
  bool coarse_inv = false;
  double *coarse_P = nullptr, *coarse_T = nullptr, *coarse_r = nullptr, *coarse_u = nullptr;
  int ld_cr = 0;
  int* status = nullptr;
  // PCG on the level-1 interface; the per-column state (vectors, partials,
  // scalars) sits in its own arena, sized for cols_cap columns
  double* partial = nullptr;
  bddc::PcgScalars* sc_host = nullptr;   // pinned, kMaxRhs columns
  bddc::Arena cols_arena;
  int cols_cap = 0;
  double* cy = nullptr;   // per column: L_II^-1 f_I (interior flat) and L_GI L_II^-1 f_I (interface flat)
  double* ct = nullptr;
  int ld_cy = 0;
  int nblk = 1;
  bddc::PcgDev pcg;
  // deep levels (2 .. L-1) and the coarsest solve in one workgroup when small
  bool fused_deep = false;
  // launch configuration (bddc_tuning): the deep path in use, PCG iterations
  // per chunk, and what the autotuner measured
  int deep_sel = BDDC_DEEP_LEVELS;
  int pcg_check = 8;
  double tuned_ms = 0.0;
  std::string shape_key;
  bddc::DeepArgs deep;
  // one deep level and the coarsest solve in one cooperative launch
  std::vector<void*> staged;   // pinned upload buffers of the setup, released after it synchronises
  bool coop_deep = false;
  bool coop_launch = false;   // use the cooperative launch API (BDDC_COOP_LAUNCH=1)
  bool coop_shared = false;   // this solve shares the device with other handles: cooperative API
  bool counted = false;       // counted in g_live_handles
  int device = 0;             // the device the handle's memory lives on
  bool noalloc_now = false;   // inside bddc_solve_noalloc: no graph, no (re)allocation
  bddc::PcgRun run;           // the solve in progress (stepwise API or a blocking solve)
  hipEvent_t run_event = nullptr;   // after the last advance's copy of the convergence flags
  int coop_rmax = 1;          // most columns one cooperative launch serves (LDS and residency)
  double coop_bytes = 0;      // algorithmic bytes of one launch
  hipGraphExec_t graph_exec = nullptr;   // one chunk of PCG launches (captured on first use)
  int graph_nrhs = 0;                    // columns of the captured chunk
  bool graph_off = false;
  bool wide_deep = false;     // one deep level in row-block launches (WideDev)
  bddc::WideDev wide;
  double wide_bytes = 0;      // algorithmic bytes of the four launches
  double wide_by[4] = {0, 0, 0, 0};   // ... of each of them (pre, restrict, coarse, post)
  bddc::Arena wide_arena;
  double by_average = 0;      // algorithmic bytes of the level-1 interface average
  double by_ur_prec = 0;      // update + restriction (it >= 1), T_rr and Psi in the precision form's storage
  double by_schur_packed = 0; // the PCG product with S_s as packed lower triangles
  double by_r_prec = 0;       // restriction of r_0 alone, likewise
  bddc::CoopDev coop;
  bddc::Arena coop_arena;
  bddc_info info{};
};

namespace bddc {

// ---------------------------------------------------------------------------
// validation
static void validate(const bddc_problem* p) {
  if (!p) fail(BDDC_EINVAL, "problem is NULL");
  if (p->nx < 2 || p->ny < 2) fail(BDDC_EINVAL, "nx and ny must be >= 2");
  if ((int64_t)p->nx * p->ny > (int64_t)1 << 30) fail(BDDC_EUNSUPPORTED, "mesh too large");
  if (p->element != BDDC_Q1 && p->element != BDDC_P1 && p->element != BDDC_Q1_ELASTIC)
    fail(BDDC_EINVAL, "unknown element");
  if ((!p->coeff && !p->coeff_device) || !p->part) fail(BDDC_EINVAL, "coeff and part are required");
  if (p->nsub < 1) fail(BDDC_EINVAL, "nsub must be >= 1");
  if (p->levels < 2 || p->levels > BDDC_MAX_LEVELS) fail(BDDC_EINVAL, "levels must be in [2, 8]");
  if (p->constraints < 0 || p->constraints > 2) fail(BDDC_EINVAL, "unknown constraint kind");

  if (std::isnan(p->tau) || p->tau < 0) fail(BDDC_EINVAL, "tau must be >= 0");
  if (p->precision != BDDC_FP64 && p->precision != BDDC_FP32 && p->precision != BDDC_BF16)
    fail(BDDC_EINVAL, "unknown precision");
  const int64_t ne = (int64_t)p->nx * p->ny;
  for (int64_t e = 0; e < ne; ++e) {
    if (!p->coeff_device) {
      const double k = p->coeff[e];
      if (!(k > 0.0) || !std::isfinite(k)) fail(BDDC_EINVAL, "coefficients must be positive and finite");
    }
    if (p->part[e] < 0 || p->part[e] >= p->nsub) fail(BDDC_EPARTITION, "partition id out of range");
  }
  std::vector<char> used(p->nsub, 0);
  for (int64_t e = 0; e < ne; ++e) used[p->part[e]] = 1;
  for (int s = 0; s < p->nsub; ++s)
    if (!used[s]) fail(BDDC_EPARTITION, "substructure " + std::to_string(s) + " owns no element");
  if (p->levels > 2) {
    if (!p->agglom) fail(BDDC_EINVAL, "agglom is required for levels > 2");
    int nprev = p->nsub;
    for (int l = 0; l < p->levels - 2; ++l) {
      const int32_t* a = p->agglom[l];
      if (!a) fail(BDDC_EINVAL, "agglom entry is NULL");
      int mx = -1;
      for (int s = 0; s < nprev; ++s) {
        if (a[s] < 0) fail(BDDC_EPARTITION, "agglomeration id out of range");
        mx = std::max(mx, a[s]);
      }
      std::vector<char> u(mx + 1, 0);
      for (int s = 0; s < nprev; ++s) u[a[s]] = 1;
      for (int g = 0; g <= mx; ++g)
        if (!u[g]) fail(BDDC_EPARTITION, "empty agglomerate");
      nprev = mx + 1;
    }
  }
}

// level-1 element -> dof incidence (Dirichlet nodes dropped)
struct Level1Elements {
  std::vector<int32_t> ptr, dof, sub;
  std::vector<uint8_t> touch;
  std::vector<int32_t> nodes;   // 4 per element, -1 = Dirichlet
};

// level-1 elements as a general element list (used by bddc_plan to check the
// grid classification against the general one)
static Level1Elements level1_elements(const bddc_problem* p) {
  const int nx = p->nx, ny = p->ny;
  Level1Elements E;
  const int ne = nx * ny;
  E.ptr.resize(ne + 1);
  E.dof.reserve((size_t)ne * 4);
  E.sub.assign(p->part, p->part + ne);
  E.touch.assign(ne, 0);
  E.nodes.resize((size_t)ne * 4);
  auto fid = [&](int i, int j) -> int {
    if (i <= 0 || j <= 0 || i >= nx || j >= ny) return -1;
    return (j - 1) * (nx - 1) + (i - 1);
  };
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int e = j * nx + i;
      const int nd[4] = {fid(i, j), fid(i + 1, j), fid(i + 1, j + 1), fid(i, j + 1)};
      E.ptr[e] = (int32_t)E.dof.size();
      for (int q = 0; q < 4; ++q) {
        E.nodes[(size_t)e * 4 + q] = nd[q];
        if (nd[q] >= 0) E.dof.push_back(nd[q]);
        else E.touch[e] = 1;
      }
    }
  E.ptr[ne] = (int32_t)E.dof.size();
  return E;
}

// ---------------------------------------------------------------------------
// host layout of a level after classification
static void layout_level(Level& lv) {
  const Topology& T = lv.topo;
  const int nsub = lv.nsub = T.nsub;
  lv.n = T.n;
  lv.koff.resize(nsub);
  std::vector<int32_t> gcnt(nsub), icnt(nsub);
  int64_t ko = 0;
  for (int s = 0; s < nsub; ++s) {
    const int n = T.nloc(s);
    lv.koff[s] = ko;
    ko += (int64_t)n * n;
    gcnt[s] = T.ngam(s);
    icnt[s] = T.n_int[s];
    lv.nImax = std::max(lv.nImax, (int)T.n_int[s]);
    lv.ngmax = std::max(lv.ngmax, T.ngam(s));
    lv.nmax = std::max(lv.nmax, n);
    lv.nrmax = std::max(lv.nrmax, (int)T.n_r[s]);
  }
  lv.goff = prefix(gcnt);
  lv.ioff = prefix(icnt);
  lv.nflat_g = lv.goff[nsub];
  lv.nflat_i = lv.ioff[nsub];
  lv.nr_v = T.n_r;
  // interface numbering (ascending dof)
  std::vector<int32_t> iid(T.n, -1);
  for (int d = 0; d < T.n; ++d)
    if (T.nshare[d] >= 2) {
      iid[d] = (int32_t)lv.iface_dof.size();
      lv.iface_dof.push_back(d);
    }
  const int nif = (int)lv.iface_dof.size();
  lv.int_gid.resize(lv.nflat_i);
  lv.gam_gid.resize(lv.nflat_g);
  lv.gam_iid.resize(lv.nflat_g);
  std::vector<int32_t> shcnt(nif, 0);
  for (int s = 0; s < nsub; ++s) {
    const int b = T.loc_ptr[s], nI = T.n_int[s], ng = T.ngam(s);
    for (int i = 0; i < nI; ++i) lv.int_gid[lv.ioff[s] + i] = T.loc_dof[b + i];
    for (int a = 0; a < ng; ++a) {
      const int d = T.loc_dof[b + nI + a];
      lv.gam_gid[lv.goff[s] + a] = d;
      lv.gam_iid[lv.goff[s] + a] = iid[d];
      shcnt[iid[d]]++;
    }
  }
  lv.sh_ptr = prefix(shcnt);
  lv.sh_flat.resize(lv.nflat_g);
  {
    std::vector<int32_t> pos(lv.sh_ptr.begin(), lv.sh_ptr.end() - 1);
    for (int s = 0; s < nsub; ++s)
      for (int a = 0; a < T.ngam(s); ++a) {
        const int f = lv.goff[s] + a;
        lv.sh_flat[pos[lv.gam_iid[f]]++] = f;
      }
  }
  // edges: shared corners then edge dofs
  lv.nedge = T.nedges();
  std::unordered_map<uint64_t, int> eid;
  eid.reserve(lv.nedge * 2 + 1);
  for (int e = 0; e < lv.nedge; ++e) eid[pkey(T.edge_s[e], T.edge_t[e])] = e;
  std::vector<std::vector<int32_t>> shared(lv.nedge);
  for (int c : T.corners)
    for (int a = 0; a < T.nshare[c]; ++a)
      for (int b2 = a + 1; b2 < T.nshare[c]; ++b2) {
        auto it = eid.find(pkey(T.share(c)[a], T.share(c)[b2]));
        if (it != eid.end()) shared[it->second].push_back(c);
      }
  lv.edge_nsc.resize(lv.nedge);
  lv.edge_ne.resize(lv.nedge);
  lv.edge_fptr.assign(1, 0);
  for (int e = 0; e < lv.nedge; ++e) {
    lv.edge_nsc[e] = (int32_t)shared[e].size();
    lv.edge_ne[e] = T.edge_ptr[e + 1] - T.edge_ptr[e];
    for (int c : shared[e]) lv.edge_fdof.push_back(c);
    for (int k = T.edge_ptr[e]; k < T.edge_ptr[e + 1]; ++k) lv.edge_fdof.push_back(T.edge_dof[k]);
    lv.edge_fptr.push_back((int32_t)lv.edge_fdof.size());
    lv.nemax = std::max(lv.nemax, (int)lv.edge_ne[e]);
    lv.nvmax = std::max(lv.nvmax, (int)(lv.edge_nsc[e] + 2 * lv.edge_ne[e]));
  }
  // incidences: 2e = s side, 2e+1 = t side
  const int ninc = 2 * lv.nedge;
  lv.inc_sub.resize(ninc);
  lv.inc_edge.resize(ninc);
  std::vector<int32_t> sic(nsub, 0);
  for (int e = 0; e < lv.nedge; ++e) {
    lv.inc_sub[2 * e] = T.edge_s[e];
    lv.inc_sub[2 * e + 1] = T.edge_t[e];
    lv.inc_edge[2 * e] = lv.inc_edge[2 * e + 1] = e;
    sic[T.edge_s[e]]++;
    sic[T.edge_t[e]]++;
  }
  lv.sub_inc_ptr = prefix(sic);
  lv.sub_inc.resize(ninc);
  {
    std::vector<int32_t> pos(lv.sub_inc_ptr.begin(), lv.sub_inc_ptr.end() - 1);
    for (int i = 0; i < ninc; ++i) lv.sub_inc[pos[lv.inc_sub[i]]++] = i;   // ascending edge per sub
  }
  lv.inc_fptr.assign(ninc + 1, 0);
  for (int i = 0; i < ninc; ++i) {
    const int e = lv.inc_edge[i];
    lv.inc_fptr[i + 1] = lv.inc_fptr[i] + (lv.edge_fptr[e + 1] - lv.edge_fptr[e]);
  }
  lv.inc_fpos.resize(lv.inc_fptr[ninc]);
  std::vector<int32_t> posin(T.n, -1);
  for (int s = 0; s < nsub; ++s) {
    const int b = T.loc_ptr[s] + T.n_int[s];
    for (int a = 0; a < T.ngam(s); ++a) posin[T.loc_dof[b + a]] = a;
    for (int k = lv.sub_inc_ptr[s]; k < lv.sub_inc_ptr[s + 1]; ++k) {
      const int i = lv.sub_inc[k], e = lv.inc_edge[i];
      int o = lv.inc_fptr[i];
      for (int q = lv.edge_fptr[e]; q < lv.edge_fptr[e + 1]; ++q) {
        const int pp = posin[lv.edge_fdof[q]];
        if (pp < 0) fail(BDDC_EPARTITION, "internal: shared dof not on the substructure interface");
        lv.inc_fpos[o++] = pp;
      }
    }
    for (int a = 0; a < T.ngam(s); ++a) posin[T.loc_dof[b + a]] = -1;
  }
  lv.inc_off.resize(ninc);
  int64_t io = 0;
  for (int i = 0; i < ninc; ++i) {
    const int nf = lv.inc_fptr[i + 1] - lv.inc_fptr[i];
    lv.inc_off[i] = io;
    io += (int64_t)nf * nf;
  }
  lv.inc_off.push_back(io);
  // workspaces (in doubles, 256-byte aligned blocks) when LDS is too small
  // (BDDC_PAIR_WS=global: always)
  auto ws_doubles = [](size_t bytes) { return (int64_t)((bytes + 255) / 256 * 32); };
  const char* wenv = getenv("BDDC_PAIR_WS");
  const bool force = wenv && std::string(wenv) == "global";
  lv.schws_off.clear();
  lv.eigws_off.clear();
  if (force || pair_schur_lds(lv.ngmax) > kLdsMax) {
    int64_t o = 0;
    for (int i = 0; i < ninc; ++i) {
      lv.schws_off.push_back(o);
      o += ws_doubles(pair_schur_lds(T.ngam(lv.inc_sub[i])));
    }
    lv.schws_off.push_back(o);
  }
  if (force || pair_eig_lds(lv.nemax, lv.nvmax) > kLdsMax) {
    int64_t o = 0;
    for (int e = 0; e < lv.nedge; ++e) {
      lv.eigws_off.push_back(o);
      o += ws_doubles(pair_eig_lds(lv.edge_ne[e], lv.edge_nsc[e] + 2 * lv.edge_ne[e]));
    }
    lv.eigws_off.push_back(o);
  }
}

// algorithmic traffic of each kernel at one level: every operator entry and
// vector entry the kernel must touch, counted once (FP64 = 8 bytes, index = 4)
static void account(Level& lv) {
  const Topology& T = lv.topo;
  double nshare_sum = 0;
  for (int g = 0; g + 1 < (int)lv.sh_ptr.size(); ++g) {
    const double m = lv.sh_ptr[g + 1] - lv.sh_ptr[g];
    nshare_sum += m * m;   // every sharer of g sums over all sharers of g
  }
  const double nif = (double)lv.iface_dof.size();
  for (int s = 0; s < lv.nsub; ++s) {
    const double nI = T.n_int[s], ng = T.ngam(s), nr = T.n_r[s], n = T.nloc(s);
    const double ncs = lv.coff[s + 1] - lv.coff[s];
    lv.by_schur += 8 * ng * ng + 20 * ng;
    lv.by_restrict_ir += 8 * nr * nr + 8 * ng * ncs + 28 * ng + 8 * ncs;
    lv.by_prolong += 8 * ng * ncs + 12 * ncs + 24 * ng;
    lv.by_pre += 8 * nI * (nI + 1) / 2 + 8 * ng * nI + 20 * nI + 8 * ng;
    lv.by_post_fs += 8 * nI * (nI + 1) / 2 + 8 * ng * nI + 20 * nI;
    for (int j = 0; j < (int)nI; ++j) {
      const double w = n - j - 1;
      lv.fl_chol += w + w * (w + 1);
    }
    lv.by_chol += 16 * n * n;
  }
  lv.by_restrict_fs = lv.by_restrict_ir + 12 * nshare_sum;
  // PCG update folded into the interface restriction: the sharers' local
  // products, r_{k-1}, and per owned dof r_k written, x read and written, p read
  lv.by_update_restrict = lv.by_restrict_ir + 12 * nshare_sum + 32 * nif;
  lv.by_post_ir = 12 * nshare_sum + 12 * lv.nflat_g + 8 * nif;
  lv.by_post_fs += lv.by_post_ir;
}

// ---------------------------------------------------------------------------
class Builder {
 public:
  Builder(bddc_ctx* h, const bddc_problem* p) : h_(h), p_(p), st_(h->stream) {}

  void run() {
    HostClock clk;
    // level 1
    GridMaps G;
    auto lv = std::make_unique<Level>();
    lv->ell = 1;
    lv->topo = classify_grid(p_->nx, p_->ny, p_->part, p_->nsub, &G);
    expand_node_topology(lv->topo, &G, dofs_per_node(p_->element));
    {
      const int dpn = dofs_per_node(p_->element);
      lv->comp.resize(lv->topo.n);
      for (int d = 0; d < lv->topo.n; ++d) lv->comp[d] = (int8_t)(d % dpn);
    }
    clk.lap("classify l1");
    layout_level(*lv);
    check_limits(*lv);
    clk.lap("layout l1");
    top_alloc();
    alloc_a(*lv, &G, nullptr);
    clk.lap("alloc_a l1");
    assemble_l1(*lv);
    factor_level(*lv, nullptr);
    clk.lap("factor l1");
    h_->levels.push_back(std::move(lv));
    for (int ell = 2; ell < h_->L; ++ell) {
      Level& prev = *h_->levels.back();
      auto nl = std::make_unique<Level>();
      nl->ell = ell;
      std::vector<int32_t> eptr(prev.nsub + 1), edof, esub(prev.agglom_of.begin(), prev.agglom_of.end());
      std::vector<uint8_t> etouch(prev.nsub);
      for (int s = 0; s < prev.nsub; ++s) {
        eptr[s] = (int32_t)edof.size();
        for (int k = prev.coff[s]; k < prev.coff[s + 1]; ++k) edof.push_back(prev.cid[k]);
        etouch[s] = prev.topo.floating[s] ? 0 : 1;
      }
      eptr[prev.nsub] = (int32_t)edof.size();
      const int nsub_next = *std::max_element(esub.begin(), esub.end()) + 1;
      nl->topo = classify(prev.nc, nsub_next, eptr, edof, esub, etouch, true);
      nl->comp = prev.cd_comp;
      layout_level(*nl);
      check_limits(*nl);
      clk.lap("classify+layout");
      alloc_a(*nl, nullptr, &prev);
      clk.lap("alloc_a");
      assemble_coarse(*nl, prev);
      factor_level(*nl, &prev);
      clk.lap("factor");
      h_->levels.push_back(std::move(nl));
    }
    coarsest();
    clk.lap("coarsest");
  }

  // Wait for the set-up's device work, release its staging buffers and check
  // the factorizations (called once everything of the set-up is enqueued).
  static void finish(bddc_ctx* h) {
    int bad = 0;
    BDDC_HIP(hipMemcpyAsync(&bad, h->status, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    BDDC_HIP(hipStreamSynchronize(h->stream));
    for (void* b : h->staged) pinned_release(b);
    h->staged.clear();
    if (bad & 2) fail(BDDC_EINVAL, "coefficients must be positive and finite");
    if (bad) fail(BDDC_ESINGULAR, "a local or coarse factorization met a non-positive pivot");
  }

 private:
  bddc_ctx* h_;
  const bddc_problem* p_;
  hipStream_t st_;

  void check_limits(const Level& lv) {
    if (partial_chol_lds(lv.nmax) > kLdsMax && !use_mfma_chol(lv.nmax) && !use_big_chol(lv.nmax))
      fail(BDDC_EUNSUPPORTED, "substructure too large for this build");
  }

  void top_alloc() {
    h_->top.reset_sizing();
    h_->status = h_->top.take<int>(1);
    h_->top.allocate(st_);
    h_->status = h_->top.take<int>(1);
    BDDC_HIP(hipMemsetAsync(h_->status, 0, sizeof(int), st_));
  }

  // device allocation of everything known before the coarse dofs are chosen
  void alloc_a(Level& lv, GridMaps* G, const Level* prev) {
    HostClock clk;
    const Topology& T = lv.topo;
    const int nsub = lv.nsub;
    const int ninc = 2 * lv.nedge;
    const bool adaptive = h_->constraints == BDDC_ADAPTIVE;
    // level-1 assembly maps (from the grid classification)
    std::vector<int32_t> node_el, sub_el_ptr, el_gid, el_loc;
    std::vector<int32_t> child_ptr, child_id, child_map_off, child_map;
    const int pe = G ? G->per_el : 4;   // element dofs in el_loc
    if (G) {
      node_el.swap(G->node_el);
      sub_el_ptr.swap(G->sub_el_ptr);
      el_gid.swap(G->el_gid);
      el_loc.swap(G->el_loc);
    }
    if (prev) {
      // children of each level-l substructure and their coarse dofs in its local numbering
      std::vector<int32_t> cnt(nsub, 0);
      for (int c = 0; c < prev->nsub; ++c) cnt[prev->agglom_of[c]]++;
      child_ptr = prefix(cnt);
      child_id.resize(prev->nsub);
      {
        std::vector<int32_t> pos(child_ptr.begin(), child_ptr.end() - 1);
        for (int c = 0; c < prev->nsub; ++c) child_id[pos[prev->agglom_of[c]]++] = c;
      }
      std::vector<int32_t> posin(T.n, -1);
      for (int s = 0; s < nsub; ++s) {
        const int b = T.loc_ptr[s];
        for (int a = 0; a < T.nloc(s); ++a) posin[T.loc_dof[b + a]] = a;
        for (int k = child_ptr[s]; k < child_ptr[s + 1]; ++k) {
          const int c = child_id[k];
          child_map_off.push_back((int32_t)child_map.size());
          for (int q = prev->coff[c]; q < prev->coff[c + 1]; ++q) child_map.push_back(posin[prev->cid[q]]);
        }
        for (int a = 0; a < T.nloc(s); ++a) posin[T.loc_dof[b + a]] = -1;
      }
    }
    // eigen work sizes
    lv.lamoff.assign(lv.nedge + 1, 0);
    lv.qoff.assign(lv.nedge + 1, 0);
    for (int e = 0; e < lv.nedge; ++e) {
      const int ne_ = lv.edge_ne[e];
      lv.lamoff[e + 1] = lv.lamoff[e] + ne_;
      lv.qoff[e + 1] = lv.qoff[e] + (int64_t)ne_ * ne_;
    }
    std::vector<int32_t> edge_ptr(T.edge_ptr), edge_dof(T.edge_dof);
    std::vector<uint8_t> floating(T.floating);
    lv.linvoff.assign(nsub + 1, 0);
    if (prev)
      for (int s = 0; s < nsub; ++s) lv.linvoff[s + 1] = lv.linvoff[s] + (int64_t)T.n_int[s] * T.n_int[s];
    // tiled elimination: per row tile of 64 local dofs (interior tiles, then
    // interface tiles) the first interior column tile of the envelope of the
    // local matrix, i.e. of its factor (fill stays right of each row's first
    // nonzero); found from the elements at level 1, every tile at other levels
    std::vector<int32_t> tproff, tprof, big_order, rgfoff, rgf;
    std::vector<int64_t> woff;
    lv.big = level_big_chol(lv.ell, lv.nmax);
    if (lv.big) {
      constexpr int kT = 64;
      tproff.assign(nsub + 1, 0);
      woff.assign(nsub + 1, 0);
      for (int s = 0; s < nsub; ++s) {
        const int nbI = (T.n_int[s] + kT - 1) / kT, nbG = (T.ngam(s) + kT - 1) / kT;
        tproff[s + 1] = tproff[s] + nbI + nbG;
        woff[s + 1] = woff[s] + (int64_t)nbI * kT * kT;
      }
      tprof.assign(tproff[nsub], 0);
      if (G) {
        rgfoff.assign(nsub + 1, 0);
        for (int s = 0; s < nsub; ++s)
          rgfoff[s + 1] = rgfoff[s] + (T.n_int[s] + 3) / 4 + (T.ngam(s) + 3) / 4;
        rgf.assign(rgfoff[nsub], 0);
      }
      if (G)
        parallel_for(nsub, 4, [&](int s0, int s1) {
          std::vector<int> f;
          for (int s = s0; s < s1; ++s) {
            const int n = T.nloc(s), nI = T.n_int[s];
            f.assign(n, INT32_MAX);
            for (int k = sub_el_ptr[s]; k < sub_el_ptr[s + 1]; ++k) {
              const int32_t* loc = &el_loc[(size_t)k * pe];
              int mn = INT32_MAX;
              for (int q = 0; q < pe; ++q)
                if (loc[q] >= 0 && loc[q] < nI) mn = std::min(mn, (int)loc[q]);
              if (mn == INT32_MAX) continue;
              for (int q = 0; q < pe; ++q)
                if (loc[q] >= 0) f[loc[q]] = std::min(f[loc[q]], mn);
            }
            const int nbI = (nI + kT - 1) / kT;
            int32_t* pr = &tprof[tproff[s]];
            for (int t = 0; t < tproff[s + 1] - tproff[s]; ++t) {
              const int r0 = t < nbI ? t * kT : nI + (t - nbI) * kT;
              const int r1 = t < nbI ? std::min(nI, r0 + kT) : std::min(n, r0 + kT);
              int mn = INT32_MAX;
              for (int r = r0; r < r1; ++r) mn = std::min(mn, f[r]);
              pr[t] = mn == INT32_MAX ? nbI : mn / kT;
            }
            // per four rows (interior, then interface): the first interior
            // column of the envelope (nI when the rows hold none)
            int32_t* gf = &rgf[rgfoff[s]];
            const int ng4 = (n - nI + 3) / 4, nI4 = (nI + 3) / 4;
            for (int g = 0; g < nI4 + ng4; ++g) {
              const int r0 = g < nI4 ? 4 * g : nI + 4 * (g - nI4);
              const int r1 = g < nI4 ? std::min(nI, r0 + 4) : std::min(n, r0 + 4);
              int mn = INT32_MAX;
              for (int r = r0; r < r1; ++r) mn = std::min(mn, f[r]);
              gf[g] = mn == INT32_MAX ? nI : mn;
            }
          }
        });
      // the substructures by decreasing envelope (tiles of the factor), the
      // order their workgroups start in (BDDC_BIG_ORDER=0: index order)
      const char* oenv = getenv("BDDC_BIG_ORDER");
      if (!(oenv && std::string(oenv) == "0")) {
        std::vector<int64_t> wgt(nsub, 0);
        for (int s = 0; s < nsub; ++s) {
          const int nbI = (T.n_int[s] + kT - 1) / kT;
          const int nt = tproff[s + 1] - tproff[s];
          for (int t = 0; t < nt; ++t) wgt[s] += std::max(0, std::min(t, nbI - 1) - tprof[tproff[s] + t] + 1);
        }
        big_order.resize(nsub);
        for (int s = 0; s < nsub; ++s) big_order[s] = s;
        std::stable_sort(big_order.begin(), big_order.end(), [&](int a, int b) { return wgt[a] > wgt[b]; });
      }
    }

    // level-1 sweeps (local matrices small enough for LDS panels): per
    // substructure and panel (64-wide panels, then 32-wide) the end of the
    // interior rows that can be nonzero in the panel's columns -- one past
    // the last interior row whose first nonzero lies left of the panel's end
    // (BDDC_SWEEP_ENV=0: every row)
    std::vector<int32_t> srendoff, srend;
    {
      const char* eenv = getenv("BDDC_SWEEP_ENV");
      const bool env_on = !(eenv && std::string(eenv) == "0");
      if (G && env_on && sweep_fits(lv.nmax)) {
        srendoff.assign(nsub + 1, 0);
        for (int s = 0; s < nsub; ++s) {
          const int nI = T.n_int[s];
          srendoff[s + 1] = srendoff[s] + (nI + 63) / 64 + (nI + 31) / 32;
        }
        srend.assign(std::max<int32_t>(1, srendoff[nsub]), 0);
        parallel_for(nsub, 8, [&](int s0, int s1) {
          std::vector<int> f;
          for (int s = s0; s < s1; ++s) {
            const int n = T.nloc(s), nI = T.n_int[s];
            f.assign(n, INT32_MAX);
            for (int k = sub_el_ptr[s]; k < sub_el_ptr[s + 1]; ++k) {
              const int32_t* loc = &el_loc[(size_t)k * pe];
              int mn = INT32_MAX;
              for (int q = 0; q < pe; ++q)
                if (loc[q] >= 0 && loc[q] < nI) mn = std::min(mn, (int)loc[q]);
              if (mn == INT32_MAX) continue;
              for (int q = 0; q < pe; ++q)
                if (loc[q] >= 0) f[loc[q]] = std::min(f[loc[q]], mn);
            }
            int32_t* e = &srend[srendoff[s]];
            for (const int bw : {64, 32}) {
              for (int b = 0; b * bw < nI; ++b) {
                const int c1 = std::min(nI, (b + 1) * bw);
                int r = c1;
                for (int i = c1; i < nI; ++i)
                  if (f[i] < c1) r = i + 1;
                *e++ = r;
              }
            }
          }
        });
      }
    }

    clk.lap("  maps");
    Arena& A = lv.arena_a;
    auto& d = lv.d;
    // the same layout runs twice: sizing (null base), then on the allocation
    auto layout = [&](bool real) {
      (void)real;
      d.loc_ptr = A.take<int32_t>(nsub + 1);
      d.nint = A.take<int32_t>(nsub);
      d.nr = A.take<int32_t>(nsub);
      d.goff = A.take<int32_t>(nsub + 1);
      d.ioff = A.take<int32_t>(nsub + 1);
      d.koff = A.take<int64_t>(nsub);
      d.int_gid = A.take<int32_t>(lv.nflat_i);
      d.gam_gid = A.take<int32_t>(lv.nflat_g);
      d.gam_iid = A.take<int32_t>(lv.nflat_g);
      d.iface_dof = A.take<int32_t>(lv.iface_dof.size());
      d.sh_ptr = A.take<int32_t>(lv.sh_ptr.size());
      d.sh_flat = A.take<int32_t>(lv.sh_flat.size());
      d.K = A.take<double>((size_t)(lv.koff.empty() ? 0 : lv.koff.back() + (int64_t)T.nloc(nsub - 1) * T.nloc(nsub - 1)));
      d.diagK = A.take<double>(lv.nflat_g);
      d.delta = A.take<double>(lv.nflat_g);
      d.node_el = A.take<int32_t>(node_el.size());
      d.sub_el_ptr = A.take<int32_t>(sub_el_ptr.size());
      d.el_gid = A.take<int32_t>(el_gid.size());
      d.el_loc = A.take<int32_t>(el_loc.size());
      d.coeff = A.take<double>(G ? (size_t)h_->nx * h_->ny : 0);
      d.child_ptr = A.take<int32_t>(child_ptr.size());
      d.child_id = A.take<int32_t>(child_id.size());
      d.child_map_off = A.take<int32_t>(child_map_off.size());
      d.child_map = A.take<int32_t>(child_map.size());
      d.inc_sub = A.take<int32_t>(ninc);
      d.inc_edge = A.take<int32_t>(ninc);
      d.inc_fptr = A.take<int32_t>(ninc + 1);
      d.inc_fpos = A.take<int32_t>(lv.inc_fpos.size());
      d.sub_inc_ptr = A.take<int32_t>(nsub + 1);
      d.sub_inc = A.take<int32_t>(ninc);
      d.edge_s = A.take<int32_t>(lv.nedge);
      d.edge_t = A.take<int32_t>(lv.nedge);
      d.edge_nsc = A.take<int32_t>(lv.nedge);
      d.edge_ne = A.take<int32_t>(lv.nedge);
      d.edge_fdof = A.take<int32_t>(lv.edge_fdof.size());
      d.edge_fptr = A.take<int32_t>(lv.edge_fptr.size());
      d.edge_ptr = A.take<int32_t>(edge_ptr.size());
      d.edge_dof = A.take<int32_t>(edge_dof.size());
      d.floating = A.take<uint8_t>(nsub);
      d.inc_off = A.take<int64_t>(lv.inc_off.size());
      d.lamoff = A.take<int64_t>(lv.lamoff.size());
      d.qoff = A.take<int64_t>(lv.qoff.size());
      d.Shat = A.take<double>(adaptive ? (size_t)lv.inc_off.back() : 0);
      d.Sff = A.take<double>(adaptive ? (size_t)lv.inc_off.back() : 0);
      d.schws_off = A.take<int64_t>(adaptive ? lv.schws_off.size() : 0);
      d.eigws_off = A.take<int64_t>(adaptive ? lv.eigws_off.size() : 0);
      d.schws = A.take<double>(adaptive && !lv.schws_off.empty() ? (size_t)lv.schws_off.back() : 0);
      d.eigws = A.take<double>(adaptive && !lv.eigws_off.empty() ? (size_t)lv.eigws_off.back() : 0);
      d.lam = A.take<double>((size_t)lv.lamoff.back());
      d.Q = A.take<double>((size_t)lv.qoff.back());
      d.nsel = A.take<int32_t>(lv.nedge);
      d.nkept = A.take<int32_t>(lv.nedge);
      d.z = A.take<double>((size_t)lv.n * h_->nz);
      d.y = A.take<double>(lv.nflat_i);
      d.t = A.take<double>(lv.nflat_g);
      d.a = A.take<double>(lv.nflat_g);
      d.v = A.take<double>(lv.nflat_g);
      d.qloc = A.take<double>(lv.nflat_g);
      d.Linv = A.take<double>((size_t)lv.linvoff[nsub]);
      d.linvoff = A.take<int64_t>(nsub + 1);
      d.tprof = A.take<int32_t>(tprof.size());
      d.tproff = A.take<int32_t>(tproff.size());
      d.rgf = A.take<int32_t>(rgf.size());
      d.rgfoff = A.take<int32_t>(rgfoff.size());
      d.Wd = A.take<double>(woff.empty() ? 0 : (size_t)woff.back());
      d.woff = A.take<int64_t>(woff.size());
      d.srend = A.take<int32_t>(srend.size());
      d.srendoff = A.take<int32_t>(srendoff.size());
      d.order = A.take<int32_t>(big_order.size());
    };
    A.reset_sizing();
    layout(false);
    A.allocate(st_);
    layout(true);
    clk.lap("  allocate");

    std::vector<int32_t> nint(T.n_int), nr(T.n_r);
    std::vector<double> ones;
    Staging stg(st_, &h_->staged);
    stg.add(d.loc_ptr, T.loc_ptr);
    stg.add(d.nint, nint);
    stg.add(d.nr, nr);
    stg.add(d.goff, lv.goff);
    stg.add(d.ioff, lv.ioff);
    stg.add(d.koff, lv.koff);
    stg.add(d.int_gid, lv.int_gid);
    stg.add(d.gam_gid, lv.gam_gid);
    stg.add(d.gam_iid, lv.gam_iid);
    stg.add(d.iface_dof, lv.iface_dof);
    stg.add(d.sh_ptr, lv.sh_ptr);
    stg.add(d.sh_flat, lv.sh_flat);
    stg.add(d.node_el, node_el);
    stg.add(d.sub_el_ptr, sub_el_ptr);
    stg.add(d.el_gid, el_gid);
    stg.add(d.el_loc, el_loc);
    if (G && p_->coeff_device)
      BDDC_HIP(hipMemcpyAsync(d.coeff, p_->coeff_device, sizeof(double) * h_->nx * h_->ny,
                              hipMemcpyDeviceToDevice, st_));
    else if (G)
      BDDC_HIP(hipMemcpyAsync(d.coeff, p_->coeff, sizeof(double) * h_->nx * h_->ny, hipMemcpyHostToDevice, st_));
    stg.add(d.child_ptr, child_ptr);
    stg.add(d.child_id, child_id);
    stg.add(d.child_map_off, child_map_off);
    stg.add(d.child_map, child_map);
    stg.add(d.inc_sub, lv.inc_sub);
    stg.add(d.inc_edge, lv.inc_edge);
    stg.add(d.inc_fptr, lv.inc_fptr);
    stg.add(d.inc_fpos, lv.inc_fpos);
    stg.add(d.sub_inc_ptr, lv.sub_inc_ptr);
    stg.add(d.sub_inc, lv.sub_inc);
    stg.add(d.edge_s, T.edge_s);
    stg.add(d.edge_t, T.edge_t);
    stg.add(d.edge_nsc, lv.edge_nsc);
    stg.add(d.edge_ne, lv.edge_ne);
    stg.add(d.edge_fdof, lv.edge_fdof);
    stg.add(d.edge_fptr, lv.edge_fptr);
    stg.add(d.edge_ptr, edge_ptr);
    stg.add(d.edge_dof, edge_dof);
    stg.add(d.floating, floating);
    stg.add(d.inc_off, lv.inc_off);
    if (lv.big) {
      stg.add(d.tprof, tprof);
      stg.add(d.tproff, tproff);
      stg.add(d.woff, woff);
      if (!rgf.empty()) {
        stg.add(d.rgf, rgf);
        stg.add(d.rgfoff, rgfoff);
      }
    }
    if (!srend.empty()) {
      stg.add(d.srend, srend);
      stg.add(d.srendoff, srendoff);
    }
    if (!big_order.empty()) stg.add(d.order, big_order);
    lv.has_order = !big_order.empty();
    lv.has_rgf = !rgf.empty() && !(getenv("BDDC_TILE_ENV") && std::string(getenv("BDDC_TILE_ENV")) == "0");
    lv.sweep_env = !srend.empty();
    if (adaptive) {
      stg.add(d.schws_off, lv.schws_off);
      stg.add(d.eigws_off, lv.eigws_off);
    }
    stg.add(d.lamoff, lv.lamoff);
    stg.add(d.qoff, lv.qoff);
    stg.add(d.linvoff, lv.linvoff);
    if (prev) {
      // the kernel modes' coarse values, computed on the previous level
      BDDC_HIP(hipMemcpyAsync(d.z, prev->d.znext, sizeof(double) * lv.n * h_->nz, hipMemcpyDeviceToDevice, st_));
    } else if (adaptive) {
      // level 1: the constants, or for elasticity the rigid-body modes at the
      // free nodes (x then y component of each node): translations x and y,
      // and the rotation u = (-y, x)
      if (h_->nz == 1) {
        ones.assign(lv.n, 1.0);
      } else {
        const int mx = h_->nx - 1;
        const int nn = lv.n / 2;
        ones.assign((size_t)lv.n * 3, 0.0);
        for (int f = 0; f < nn; ++f) {
          const double x = (double)(f % mx + 1) / h_->nx, y = (double)(f / mx + 1) / h_->ny;
          ones[2 * f] = 1.0;
          ones[(size_t)lv.n + 2 * f + 1] = 1.0;
          ones[2 * (size_t)lv.n + 2 * f] = -y;
          ones[2 * (size_t)lv.n + 2 * f + 1] = x;
        }
      }
      stg.add(d.z, ones);
    }
    stg.flush();
    clk.lap("  staging");
    // the staging buffer waits for its copies when it goes out of scope
  }

  void assemble_l1(Level& lv) {
    if (p_->element == BDDC_Q1_ELASTIC) {
      const Khat64 kh = elastic_element_matrix(h_->nx, h_->ny);
      launch_assemble_l1_elastic(st_, lv.nsub, lv.d.koff, lv.d.loc_ptr, lv.d.nint, lv.d.node_el, lv.d.sub_el_ptr,
                                 lv.d.el_gid, lv.d.el_loc, lv.d.coeff, kh, lv.d.K, lv.d.diagK, lv.d.goff,
                                 h_->status);
      return;
    }
    const Khat16 kh = element_matrix(p_->element, h_->nx, h_->ny);
    launch_assemble_l1(st_, lv.nsub, lv.d.koff, lv.d.loc_ptr, lv.d.nint, lv.d.node_el, lv.d.sub_el_ptr,
                       lv.d.el_gid, lv.d.el_loc, lv.d.coeff, kh, lv.d.K, lv.d.diagK, lv.d.goff, h_->status);
  }

  void assemble_coarse(Level& lv, const Level& prev) {
    launch_assemble_coarse(st_, lv.nsub, lv.d.koff, lv.d.loc_ptr, lv.d.nint, lv.d.child_ptr, lv.d.child_id,
                           lv.d.child_map_off, lv.d.child_map, prev.d.Ac, prev.d.acoff, prev.d.ncs, lv.d.K,
                           lv.d.diagK, lv.d.goff);
  }

  // weights, interior elimination, constraint selection, constrained factors
  void factor_level(Level& lv, const Level*) {
    HostClock clk;
    auto& d = lv.d;
    const Topology& T = lv.topo;
    launch_weights(st_, lv.nflat_g, d.gam_iid, d.sh_ptr, d.sh_flat, d.diagK, d.delta);
    {
      double fl = 0;
      for (int s = 0; s < lv.nsub; ++s)
        for (int j = 0; j < T.n_int[s]; ++j) {
          const double w = T.nloc(s) - j - 1;
          fl += w + w * (w + 1);
        }
      double by = 0;
      for (int s = 0; s < lv.nsub; ++s) by += 16.0 * T.nloc(s) * T.nloc(s);
      timing::Scope ts(lv.ell == 1 ? "partial_chol" : "partial_chol_l2", by, fl);
      if (lv.big) {
        LevelDev D{};
        D.nsub = lv.nsub;
        D.koff = d.koff;
        D.loc_ptr = d.loc_ptr;
        D.nint = d.nint;
        D.tprof = d.tprof;
        D.tproff = d.tproff;
        D.woff = d.woff;
        D.order = lv.has_order ? d.order : nullptr;
        launch_partial_chol_big(st_, D, d.K, d.Wd, h_->status);
      }
      else if (use_mfma_chol(lv.nmax))
        launch_partial_chol_mfma(st_, lv.nsub, lv.nmax, d.koff, d.loc_ptr, d.nint, d.K, h_->status);
      else
        launch_partial_chol(st_, lv.nsub, lv.nmax, d.koff, d.loc_ptr, d.nint, d.K, h_->status);
    }
    if (lv.ell >= 2) {
      if (use_lds_setup() && tri_inverse_lds(lv.nImax) <= kLdsMax)
        launch_tri_inverse_lds(st_, lv.nsub, lv.nImax, d.koff, d.loc_ptr, d.nint, d.K, d.Linv, d.linvoff);
      else
        launch_tri_inverse(st_, lv.nsub, lv.nImax, d.koff, d.loc_ptr, d.nint, d.K, d.Linv, d.linvoff);
    }
    const int ne_tot = lv.nedge;
    lv.edge_m.assign(ne_tot, 0);
    lv.edge_nsel.assign(ne_tot, 0);
    std::vector<double> qh;
    if (h_->constraints == BDDC_ADAPTIVE && ne_tot > 0 && h_->nz > 1) {
      // elasticity: the pair problems regularise only the rigid-body modes
      // common to both substructures, so an edge of a floating substructure
      // must end at two corner nodes (which fix the relative rigid motion),
      // as on square partitions
      for (int e = 0; e < ne_tot; ++e)
        if ((T.floating[T.edge_s[e]] || T.floating[T.edge_t[e]]) && lv.edge_nsc[e] < 4)
          fail(BDDC_EUNSUPPORTED, "elasticity with adaptive constraints: an edge of a floating substructure "
                                  "shares fewer than two corner nodes");
    }
    if (h_->constraints == BDDC_ADAPTIVE && ne_tot > 0) {
      launch_pair_schur(st_, 2 * ne_tot, lv.ngmax, d.inc_sub, d.inc_fptr, d.inc_fpos, d.koff, d.loc_ptr, d.nint,
                        d.K, d.inc_off, d.Shat, d.Sff, h_->status, lv.schws_off.empty() ? nullptr : d.schws,
                        d.schws_off);
      launch_pair_eig(st_, ne_tot, lv.nemax, lv.nvmax, d.edge_s, d.edge_t, d.edge_nsc, d.edge_ne, d.edge_fdof,
                      d.edge_fptr, d.inc_fptr, d.inc_fpos, d.goff, d.diagK, d.floating, d.z, h_->nz, lv.n, d.Shat,
                      d.Sff,
                      d.inc_off, h_->tau, d.lam, d.lamoff, d.Q, d.qoff, d.nsel, d.nkept, h_->status,
                      lv.eigws_off.empty() ? nullptr : d.eigws, d.eigws_off);
      std::vector<int32_t> nkept(ne_tot);
      lv.lam.resize(lv.lamoff.back());
      {
        // one pinned buffer, so the three copies are asynchronous and one wait covers them
        const size_t bl = sizeof(double) * lv.lam.size(), bi = sizeof(int32_t) * (size_t)ne_tot;
        char* pin = static_cast<char*>(pinned_acquire(bl + 2 * bi + 16));
        BDDC_HIP(hipMemcpyAsync(pin, d.lam, bl, hipMemcpyDeviceToHost, st_));
        BDDC_HIP(hipMemcpyAsync(pin + bl, d.nkept, bi, hipMemcpyDeviceToHost, st_));
        BDDC_HIP(hipMemcpyAsync(pin + bl + bi, d.nsel, bi, hipMemcpyDeviceToHost, st_));
        clk.lap("  enqueue factor+eig");
        const hipError_t we = hipStreamSynchronize(st_);
        if (we == hipSuccess) {
          std::memcpy(lv.lam.data(), pin, bl);
          std::memcpy(nkept.data(), pin + bl, bi);
          std::memcpy(lv.edge_nsel.data(), pin + bl + bi, bi);
        }
        pinned_release(pin);
        BDDC_HIP(we);
      }
      clk.lap("  wait eig");
      lv.omega = 0.0;
      for (int e = 0; e < ne_tot; ++e) {
        lv.edge_m[e] = nkept[e];
        lv.n_adaptive += nkept[e];
        const int ns = lv.edge_nsel[e], nn = lv.edge_ne[e];
        const double nxt = ns < nn ? lv.lam[lv.lamoff[e] + ns] : 0.0;
        lv.omega = std::max(lv.omega, nxt);
      }
    } else if (h_->constraints == BDDC_CORNERS_EDGES && ne_tot > 0) {
      // the arithmetic average over the edge of each displacement component
      // present on it (Table 1: two per edge in 2D elasticity), components in
      // increasing order; column j of the edge's Q at stride edge_ne
      qh.assign(lv.qoff.back(), 0.0);
      lv.edge_ccomp.assign((size_t)ne_tot * kMaxComp, 0);
      for (int e = 0; e < ne_tot; ++e) {
        const int nn = lv.edge_ne[e];
        const int32_t* dof = T.edge_dof.data() + T.edge_ptr[e];
        int cnt[kMaxComp] = {};
        for (int p = 0; p < nn; ++p) cnt[lv.comp[dof[p]] + 1]++;
        int m = 0;
        for (int c = 0; c < kMaxComp; ++c) {
          if (!cnt[c]) continue;
          for (int p = 0; p < nn; ++p)
            if (lv.comp[dof[p]] + 1 == c) qh[lv.qoff[e] + (size_t)m * nn + p] = 1.0 / cnt[c];
          lv.edge_ccomp[(size_t)e * kMaxComp + m] = (int8_t)(c - 1);
          ++m;
        }
        lv.edge_m[e] = m;
      }
      h2d(d.Q, qh, st_);
    }
    coarse_numbering(lv);
    clk.lap("  coarse numbering");
    account(lv);
    clk.lap("  account");
    alloc_b(lv);
    clk.lap("  alloc_b");
    launch_build_cr(st_, lv.nsub, d.sub_inc_ptr, d.sub_inc, d.inc_edge, d.inc_fptr, d.inc_fpos, d.edge_nsc,
                    d.edge_ne, d.edge_m, d.qoff, d.Q, d.nr, d.ncr, d.croff, d.Cr);
    size_t cf_lds = 0;
    for (int s = 0; s < lv.nsub; ++s)
      cf_lds = std::max(cf_lds, constrained_factor_lds(T.ngam(s), T.n_r[s], lv.ncr[s], lv.coff[s + 1] - lv.coff[s]));
    if (use_lds_setup() && cf_lds <= kLdsMax)
      launch_constrained_factor_lds(st_, lv.nsub, cf_lds, d.koff, d.loc_ptr, d.nint, d.nr, d.ncr, d.croff, d.Cr,
                                    d.K, d.T, d.toff, d.Psi, d.psioff, d.Ac, d.acoff, h_->status);
    else
      launch_constrained_factor(st_, lv.nsub, d.koff, d.loc_ptr, d.nint, d.nr, d.ncr, d.croff, d.Cr, d.K, d.T,
                                d.toff, d.Psi, d.psioff, d.Ac, d.acoff, d.cwork, d.cwoff, h_->status);
    if (h_->constraints == BDDC_ADAPTIVE && lv.ell < h_->L - 1)
      launch_coarse_z(st_, lv.nc, d.cd_dof, d.cd_col, d.edge_ptr, d.edge_dof, d.qoff, d.Q, d.z, h_->nz, lv.n,
                      d.znext);
    (void)T;
    // agglomeration towards the next level
    if (lv.ell < h_->L - 1) {
      const int32_t* a = p_->agglom[lv.ell - 1];
      lv.agglom_of.assign(a, a + lv.nsub);
    }
    fill_dev(lv);
  }

  void coarse_numbering(Level& lv) {
    const Topology& T = lv.topo;
    const int nsub = lv.nsub;
    const int ncorner = (int)T.corners.size();
    std::vector<int32_t> corner_id(T.n, -1);
    for (int k = 0; k < ncorner; ++k) corner_id[T.corners[k]] = k;
    std::vector<int32_t> ebase(lv.nedge + 1, ncorner);
    for (int e = 0; e < lv.nedge; ++e) ebase[e + 1] = ebase[e] + lv.edge_m[e];
    lv.nc = ebase[lv.nedge];
    lv.cd_dof.resize(lv.nc);
    lv.cd_col.resize(lv.nc);
    lv.cd_comp.resize(lv.nc);
    for (int k = 0; k < ncorner; ++k) {
      lv.cd_dof[k] = T.corners[k];
      lv.cd_col[k] = -1;
      lv.cd_comp[k] = lv.comp[T.corners[k]];
    }
    const bool averages = !lv.edge_ccomp.empty();
    for (int e = 0; e < lv.nedge; ++e)
      for (int j = 0; j < lv.edge_m[e]; ++j) {
        lv.cd_dof[ebase[e] + j] = e;
        lv.cd_col[ebase[e] + j] = j;
        lv.cd_comp[ebase[e] + j] = averages ? lv.edge_ccomp[(size_t)e * kMaxComp + j] : (int8_t)-1;
      }
    std::vector<int32_t> cnt(nsub);
    lv.ncr.assign(nsub, 0);
    for (int s = 0; s < nsub; ++s) {
      for (int k = lv.sub_inc_ptr[s]; k < lv.sub_inc_ptr[s + 1]; ++k) lv.ncr[s] += lv.edge_m[lv.inc_edge[lv.sub_inc[k]]];
      cnt[s] = T.n_c[s] + lv.ncr[s];
    }
    lv.coff = prefix(cnt);
    lv.nflat_c = lv.coff[nsub];
    lv.cid.resize(lv.nflat_c);
    std::vector<int32_t> ccnt(lv.nc, 0);
    for (int s = 0; s < nsub; ++s) {
      int o = lv.coff[s];
      const int b = T.loc_ptr[s] + T.n_int[s] + T.n_r[s];
      for (int k = 0; k < T.n_c[s]; ++k) lv.cid[o++] = corner_id[T.loc_dof[b + k]];
      for (int k = lv.sub_inc_ptr[s]; k < lv.sub_inc_ptr[s + 1]; ++k) {
        const int e = lv.inc_edge[lv.sub_inc[k]];
        for (int j = 0; j < lv.edge_m[e]; ++j) lv.cid[o++] = ebase[e] + j;
      }
      lv.ncsmax = std::max(lv.ncsmax, cnt[s]);
    }
    for (int k : lv.cid) ccnt[k]++;
    lv.csh_ptr = prefix(ccnt);
    lv.csh_flat.resize(lv.nflat_c);
    {
      std::vector<int32_t> pos(lv.csh_ptr.begin(), lv.csh_ptr.end() - 1);
      for (int f = 0; f < lv.nflat_c; ++f) lv.csh_flat[pos[lv.cid[f]]++] = f;
    }
    // per-substructure offsets of constrained-factor data
    lv.croff.assign(nsub + 1, 0);
    lv.toff.assign(nsub + 1, 0);
    lv.psioff.assign(nsub + 1, 0);
    lv.acoff.assign(nsub + 1, 0);
    lv.cwoff.assign(nsub + 1, 0);
    for (int s = 0; s < nsub; ++s) {
      const int64_t nr = T.n_r[s], ng = T.ngam(s), ncr = lv.ncr[s], ncs = cnt[s];
      lv.croff[s + 1] = lv.croff[s] + ncr * nr;
      lv.toff[s + 1] = lv.toff[s] + nr * nr;
      lv.psioff[s + 1] = lv.psioff[s] + ng * ncs;
      lv.acoff[s + 1] = lv.acoff[s] + ncs * ncs;
      lv.cwoff[s + 1] = lv.cwoff[s] + nr * nr + 2 * nr * ncr + ncr * ncr + ng * ncs;
    }
  }

  void alloc_b(Level& lv) {
    Arena& A = lv.arena_b;
    auto& d = lv.d;
    const int nsub = lv.nsub;
    const bool last = lv.ell == h_->L - 1;
    auto layout = [&]() {
      d.edge_m = A.take<int32_t>(lv.nedge);
      d.coff = A.take<int32_t>(nsub + 1);
      d.cid = A.take<int32_t>(lv.nflat_c);
      d.csh_ptr = A.take<int32_t>(lv.nc + 1);
      d.csh_flat = A.take<int32_t>(lv.nflat_c);
      d.cd_dof = A.take<int32_t>(lv.nc);
      d.cd_col = A.take<int32_t>(lv.nc);
      d.ncr = A.take<int32_t>(nsub);
      d.ncs = A.take<int32_t>(nsub);
      d.croff = A.take<int64_t>(nsub + 1);
      d.toff = A.take<int64_t>(nsub + 1);
      d.psioff = A.take<int64_t>(nsub + 1);
      d.acoff = A.take<int64_t>(nsub + 1);
      d.cwoff = A.take<int64_t>(nsub + 1);
      d.Cr = A.take<double>(lv.croff[nsub]);
      d.T = A.take<double>(lv.toff[nsub]);
      d.Psi = A.take<double>(lv.psioff[nsub]);
      d.Ac = A.take<double>(lv.acoff[nsub]);
      d.cwork = A.take<double>(lv.cwoff[nsub]);
      d.znext = A.take<double>((size_t)lv.nc * h_->nz);
      d.b = A.take<double>(lv.nflat_c);
      d.rc = A.take<double>(lv.nc);
      d.uc = A.take<double>(lv.nc);
      if (last) {
        const char* cenv = getenv("BDDC_COARSE");
        h_->coarse_inv = lv.nc >= kCoarseInvMin || (cenv && std::string(cenv) == "inverse");
        h_->AL = A.take<double>((size_t)lv.nc * lv.nc);
        if (h_->coarse_inv) {
          h_->ld_cr = (int)(((std::max(lv.nc, 1) * 8 + 255) / 256) * 32);
          h_->coarse_P = A.take<double>(64 * 64);
          h_->coarse_T = A.take<double>((size_t)std::max(lv.nc, 1) * 64);
          h_->coarse_r = A.take<double>((size_t)kMaxRhs * h_->ld_cr);
          h_->coarse_u = A.take<double>((size_t)kMaxRhs * h_->ld_cr);
        }
      }
    };
    A.reset_sizing();
    layout();
    A.allocate(st_);
    layout();
    Staging stg(st_, &h_->staged);
    stg.add(d.edge_m, lv.edge_m);
    stg.add(d.coff, lv.coff);
    stg.add(d.cid, lv.cid);
    stg.add(d.csh_ptr, lv.csh_ptr);
    stg.add(d.csh_flat, lv.csh_flat);
    stg.add(d.cd_dof, lv.cd_dof);
    stg.add(d.cd_col, lv.cd_col);
    stg.add(d.ncr, lv.ncr);
    std::vector<int32_t> ncs(nsub);
    for (int s = 0; s < nsub; ++s) ncs[s] = lv.coff[s + 1] - lv.coff[s];
    stg.add(d.ncs, ncs);
    stg.add(d.croff, lv.croff);
    stg.add(d.toff, lv.toff);
    stg.add(d.psioff, lv.psioff);
    stg.add(d.acoff, lv.acoff);
    stg.add(d.cwoff, lv.cwoff);
    stg.flush();
  }

  void fill_dev(Level& lv) {
    LevelDev& D = lv.dev;
    auto& d = lv.d;
    D.nsub = lv.nsub;
    D.nc = lv.nc;
    D.koff = d.koff;
    D.loc_ptr = d.loc_ptr;
    D.nint = d.nint;
    D.nr = d.nr;
    D.goff = d.goff;
    D.ioff = d.ioff;
    D.coff = d.coff;
    D.int_gid = d.int_gid;
    D.gam_gid = d.gam_gid;
    D.gam_iid = d.gam_iid;
    D.sh_ptr = d.sh_ptr;
    D.sh_flat = d.sh_flat;
    D.cid = d.cid;
    D.K = d.K;
    D.delta = d.delta;
    D.T = d.T;
    D.toff = d.toff;
    D.Psi = d.Psi;
    D.psioff = d.psioff;
    D.Linv = d.Linv;
    D.linvoff = d.linvoff;
    D.tprof = lv.big ? d.tprof : nullptr;
    D.tproff = lv.big ? d.tproff : nullptr;
    D.rgf = lv.big && lv.has_rgf ? d.rgf : nullptr;
    D.rgfoff = lv.big && lv.has_rgf ? d.rgfoff : nullptr;
    D.srend = lv.sweep_env ? d.srend : nullptr;
    D.srendoff = lv.sweep_env ? d.srendoff : nullptr;
    D.order = lv.has_order ? d.order : nullptr;
    D.Wd = lv.big ? d.Wd : nullptr;
    D.woff = lv.big ? d.woff : nullptr;
    D.csh_ptr = d.csh_ptr;
    D.csh_flat = d.csh_flat;
    D.y = d.y;
    D.t = d.t;
    D.a = d.a;
    D.v = d.v;
    D.b = d.b;
  }

  void coarsest() {
    Level& lv = *h_->levels.back();
    h_->ncL = lv.nc;
    if (lv.nc > 0 && h_->coarse_inv) {
      launch_coarsest_assemble(st_, lv.nsub, lv.nc, lv.d.coff, lv.d.cid, lv.d.Ac, lv.d.acoff, h_->AL);
      launch_coarsest_inverse(st_, lv.nc, h_->AL, h_->coarse_P, h_->coarse_T, h_->status);
    } else if (lv.nc > 0) {
      launch_coarsest_factor(st_, lv.nsub, lv.nc, lv.d.coff, lv.d.cid, lv.d.Ac, lv.d.acoff, h_->AL, h_->status);
    }
  }
};

// ---------------------------------------------------------------------------
// apply: Algorithm "Multilevel BDDC"
//
// Levels >= 2 run in full space with the explicit inverse of their interior
// factors; level 1 runs in full space for bddc_apply and on the interface
// inside bddc_solve.
// u_L = A_L^-1 r_L: two triangular solves with the Cholesky factor in one
// workgroup, or the product with A_L^-1 for a large coarse space
static void coarsest_solve(bddc_ctx* h, hipStream_t st, int nc, const double* rc, double* uc, const int32_t* stop) {
  if (h->coarse_inv)
    launch_coarse_inv_apply(st, nc, h->AL, rc, nc, uc, nc, 1, stop);
  else
    launch_coarsest_solve(st, nc, h->AL, rc, uc, stop);
}

static void apply_deep_level(bddc_ctx* h, int li, const double* r, double* u, hipStream_t st) {
  Level& lv = *h->levels[li];
  const std::string sfx = "_l" + std::to_string(li + 1);
  {
    timing::Scope ts(("apply_pre" + sfx).c_str(), lv.by_pre, 0);
    launch_apply_pre_inv(st, lv.dev, lv.nImax, lv.ngmax, r);
  }
  {
    timing::Scope ts(("apply_restrict" + sfx).c_str(), lv.by_restrict_fs, 0);
    launch_apply_restrict(st, lv.dev, lv.ngmax, r, lv.d.gam_gid, 1);
  }
  launch_coarse_gather(st, lv.nc, lv.d.csh_ptr, lv.d.csh_flat, lv.d.b, lv.d.rc, lv.dev.stop);
  if (li + 1 == (int)h->levels.size())
    coarsest_solve(h, st, lv.nc, lv.d.rc, lv.d.uc, lv.dev.stop);
  else
    apply_deep_level(h, li + 1, lv.d.rc, lv.d.uc, st);
  {
    timing::Scope ts(("apply_prolong" + sfx).c_str(), lv.by_prolong, 0);
    launch_apply_prolong(st, lv.dev, lv.ncsmax, lv.d.uc);
  }
  {
    timing::Scope ts(("apply_post" + sfx).c_str(), lv.by_post_fs, 0);
    launch_apply_post_inv(st, lv.dev, lv.nImax, lv.ngmax, u);
  }
}

// the four launches of the row-block deep level, each timed under its own name
static void wide_launches(bddc_ctx* h, hipStream_t st, const WideDev& W, const int32_t* gam_gid2) {
  {
    timing::Scope ts("wide_pre", h->wide_by[0], 0);
    launch_wide_pre(st, W);
  }
  {
    timing::Scope ts("wide_restrict", h->wide_by[1], 0);
    launch_wide_restrict(st, W, gam_gid2);
  }
  {
    timing::Scope ts("wide_coarse", h->wide_by[2], 0);
    launch_wide_coarse(st, W);
  }
  {
    timing::Scope ts("wide_post", h->wide_by[3], 0);
    launch_wide_post(st, W);
  }
}

// level-1 coarse right-hand side (the level-1 b) -> level-1 coarse solution (level-1 uc)
// Levels >= 2 and the coarsest solve for the level-1 coarse contributions b1
// (local coarse flat), leaving the level-1 coarse correction in uc.
static void run_deep_at(bddc_ctx* h, hipStream_t st, const double* b1, double* uc) {
  Level& l1 = *h->levels[0];
  if (h->levels.size() == 1) {
    launch_coarse_gather(st, l1.nc, l1.d.csh_ptr, l1.d.csh_flat, b1, l1.d.rc, l1.dev.stop);
    coarsest_solve(h, st, l1.nc, l1.d.rc, uc, l1.dev.stop);
    return;
  }
  if (h->deep_sel == BDDC_DEEP_COOP) {
    CoopDev C = h->coop;
    C.stop = l1.dev.stop;
    C.b1 = b1;
    C.u2 = uc;
    timing::Scope ts("deep", h->coop_bytes, 0);
    launch_deep_coop(st, C, h->coop_launch || h->coop_shared);
    return;
  }
  if (h->deep_sel == BDDC_DEEP_WIDE) {
    Level& l2 = *h->levels[1];
    WideDev W = h->wide;
    W.b1 = b1;
    W.u2 = uc;
    W.nrhs = 1;
    W.stop = l1.dev.stop;
    W.L.stop = l1.dev.stop;
    wide_launches(h, st, W, l2.d.gam_gid);
    return;
  }
  if (h->deep_sel == BDDC_DEEP_FUSED) {
    DeepArgs A = h->deep;
    A.stop = l1.dev.stop;
    A.b1 = b1;
    A.uvec[0] = uc;
    timing::Scope ts("deep", 0, 0);
    launch_deep(st, A);
    return;
  }
  launch_coarse_gather(st, l1.nc, l1.d.csh_ptr, l1.d.csh_flat, b1, l1.d.rc, l1.dev.stop);
  apply_deep_level(h, 1, l1.d.rc, uc, st);
}

static void run_deep(bddc_ctx* h, hipStream_t st) {
  Level& l1 = *h->levels[0];
  run_deep_at(h, st, l1.d.b, l1.d.uc);
}

// The deep levels for R columns of b1 / uc (strides ldb, ldu): one
// cooperative launch for all of them when it fits, else column by column.
// With rr, the level-1 r.r sums of the PCG columns may be formed by the deep
// launches themselves (the wide path's pre kernel); returns whether they were.
static bool run_deep_cols(bddc_ctx* h, hipStream_t st, const double* b1, int ldb, double* uc, int ldu, int R,
                          const PcgDev* rr = nullptr) {
  Level& l1 = *h->levels[0];
  if (h->levels.size() == 1) {
    if (h->coarse_inv) {
      launch_coarse_gather_cols(st, l1.nc, l1.d.csh_ptr, l1.d.csh_flat, b1, ldb, h->coarse_r, h->ld_cr, R,
                                l1.dev.stop);
      launch_coarse_inv_apply(st, l1.nc, h->AL, h->coarse_r, h->ld_cr, uc, ldu, R, l1.dev.stop);
    } else {
      launch_coarse_direct_cols(st, l1.nc, l1.d.csh_ptr, l1.d.csh_flat, b1, ldb, h->AL, uc, ldu, R, l1.dev.stop);
    }
    return false;
  }
  if (h->deep_sel == BDDC_DEEP_WIDE && R <= kMaxRhs) {
    Level& l2 = *h->levels[1];
    WideDev W = h->wide;
    W.nrhs = R;
    W.b1 = b1;
    W.ld_b1 = ldb;
    W.u2 = uc;
    W.ld_u2 = ldu;
    W.stop = l1.dev.stop;
    W.L.stop = l1.dev.stop;
    if (rr) {
      W.sc = rr->sc;
      W.rr_part = rr->rr_part;
      W.rr_ld = rr->ld_sub;
      W.rr_n = rr->nsub1;
    }
    wide_launches(h, st, W, l2.d.gam_gid);
    return rr != nullptr;
  }
  if (h->deep_sel == BDDC_DEEP_COOP && R <= h->coop_rmax) {
    CoopDev C = h->coop;
    C.stop = h->levels[0]->dev.stop;
    C.nrhs = R;
    C.b1 = b1;
    C.ld_b1 = ldb;
    C.u2 = uc;
    C.ld_u2 = ldu;
    timing::Scope ts("deep", h->coop_bytes, 0);
    launch_deep_coop(st, C, h->coop_launch || h->coop_shared);
    return false;
  }
  for (int c = 0; c < R; ++c) run_deep_at(h, st, b1 + (size_t)c * ldb, uc + (size_t)c * ldu);
  return false;
}

// full-space preconditioner of the level-1 problem (bddc_apply)
static void apply_full(bddc_ctx* h, const double* r, double* u) {
  Level& l1 = *h->levels[0];
  hipStream_t st = h->stream;
  const bool sweep = use_sweep(l1.nmax);
  if (sweep)
    launch_sweep_pre(st, l1.dev, r);
  else
    launch_apply_pre(st, l1.dev, l1.nImax, l1.ngmax, r);
  launch_apply_restrict(st, l1.dev, l1.ngmax, r, l1.d.gam_gid, 1);
  {
    // bddc_apply returns before its kernels run, so it could not report a
    // grid barrier that timed out: the deep levels take a path without grid
    // barriers here (the row-block path, else one launch per phase)
    struct Restore {
      bddc_ctx* h;
      int sel;
      ~Restore() { h->deep_sel = sel; }
    } restore{h, h->deep_sel};
    if (h->deep_sel == BDDC_DEEP_COOP) h->deep_sel = h->wide_deep ? BDDC_DEEP_WIDE : BDDC_DEEP_LEVELS;
    run_deep(h, st);
  }
  launch_apply_prolong(st, l1.dev, l1.ncsmax, l1.d.uc);
  if (sweep)
    launch_sweep_post(st, l1.dev, u, l1.d.gam_gid);
  else
    launch_apply_post(st, l1.dev, l1.nImax, l1.ngmax, u, l1.d.gam_gid, 1);
}

// One deep level and a small coarsest problem: pack the level-2 operators and
// index lists per substructure and use the cooperative kernel if it fits.
static bool plan_coop(bddc_ctx* h) {
  h->coop_deep = false;
  if (h->levels.size() != 2 || h->coarse_inv) return false;
  const char* env = getenv("BDDC_DEEP_PATH");
  if (env && std::string(env) != "coop") return false;
  Level& l1 = *h->levels[0];
  Level& lv = *h->levels[1];
  const Topology& T = lv.topo;
  const int nsub = lv.nsub;
  const int ncL = lv.nc;
  if (ncL < 1 || nsub < 1) return false;
  if (sizeof(double) * ((size_t)ncL * ncL + 2 * (size_t)ncL) > kLdsMax) return false;
  CoopDev C{};
  C.nsub = nsub;
  C.ncL = ncL;
  std::vector<int32_t> meta((size_t)kCoopMeta * nsub);
  std::vector<int64_t> opoff(nsub + 1, 0), idxoff(nsub + 1, 0);
  std::vector<int32_t> idx;
  std::vector<int32_t> sub_of_flat(lv.nflat_g);
  for (int s = 0; s < nsub; ++s)
    for (int f = lv.goff[s]; f < lv.goff[s + 1]; ++f) sub_of_flat[f] = s;
  for (int s = 0; s < nsub; ++s) {
    const int nI = T.n_int[s], ng = T.ngam(s), nr = T.n_r[s], ncs = lv.coff[s + 1] - lv.coff[s];
    const size_t i0 = idx.size();
    for (int i = 0; i < nI; ++i) idx.push_back(lv.int_gid[lv.ioff[s] + i]);
    for (int a = 0; a < ng; ++a) idx.push_back(lv.gam_gid[lv.goff[s] + a]);
    for (int a = 0; a < ng; ++a) {
      const int f = lv.goff[s] + a, gi = lv.gam_iid[f];
      idx.push_back(lv.sh_flat[lv.sh_ptr[gi]] == f ? 1 : 0);
    }
    std::vector<int32_t> shp(ng + 1, 0), shf;
    for (int a = 0; a < ng; ++a) {
      const int gi = lv.gam_iid[lv.goff[s] + a];
      for (int k = lv.sh_ptr[gi]; k < lv.sh_ptr[gi + 1]; ++k) shf.push_back(lv.sh_flat[k]);
      shp[a + 1] = (int32_t)shf.size();
    }
    idx.insert(idx.end(), shp.begin(), shp.end());
    idx.insert(idx.end(), shf.begin(), shf.end());
    const int n = nI + ng;
    std::vector<int32_t> gp(n + 1, 0), gf;
    for (int p = 0; p < n; ++p) {
      const int k = p < nI ? lv.int_gid[lv.ioff[s] + p] : lv.gam_gid[lv.goff[s] + p - nI];
      for (int q = l1.csh_ptr[k]; q < l1.csh_ptr[k + 1]; ++q) gf.push_back(l1.csh_flat[q]);
      gp[p + 1] = (int32_t)gf.size();
    }
    idx.insert(idx.end(), gp.begin(), gp.end());
    idx.insert(idx.end(), gf.begin(), gf.end());
    for (int k = lv.coff[s]; k < lv.coff[s + 1]; ++k) idx.push_back(lv.cid[k]);
    // rows of the delta-weighted coarse basis of all sharers of each interface dof
    std::vector<int32_t> phi_ptr(ng + 1, 0), phi_ids;
    for (int a = 0; a < ng; ++a) {
      for (int q = shp[a]; q < shp[a + 1]; ++q) {
        const int t = sub_of_flat[shf[q]];
        for (int k = lv.coff[t]; k < lv.coff[t + 1]; ++k) phi_ids.push_back(lv.cid[k]);
      }
      phi_ptr[a + 1] = (int32_t)phi_ids.size();
    }
    idx.insert(idx.end(), phi_ptr.begin(), phi_ptr.end());
    idx.insert(idx.end(), phi_ids.begin(), phi_ids.end());
    idxoff[s + 1] = (int64_t)idx.size();
    int32_t* m = meta.data() + (size_t)kCoopMeta * s;
    m[0] = nI;
    m[1] = ng;
    m[2] = nr;
    m[3] = ncs;
    m[4] = (int32_t)shf.size();
    m[5] = (int32_t)gf.size();
    m[6] = lv.goff[s];
    m[7] = lv.coff[s];
    m[8] = (int32_t)phi_ids.size();
    const int64_t ops = (int64_t)nI * nI + (int64_t)ng * nI + (int64_t)nr * nr + (int64_t)ng * ncs + ng +
                        (int64_t)phi_ids.size();
    opoff[s + 1] = opoff[s] + ops;
    C.opmax = std::max<int>(C.opmax, (int)ops);
    C.idxmax = std::max<int>(C.idxmax, (int)(idx.size() - i0));
    C.nImax = std::max(C.nImax, nI);
    C.ngmax = std::max(C.ngmax, ng);
    C.ncsmax = std::max(C.ncsmax, ncs);
  }
  std::vector<int32_t> cg(lv.csh_ptr.begin(), lv.csh_ptr.end());
  cg.insert(cg.end(), lv.csh_flat.begin(), lv.csh_flat.end());
  C.cg_len = (int)cg.size();
  const size_t lds = coop_lds(C);
  if (lds > kLdsMax) return false;
  if (coop_max_blocks(lds) < nsub) return false;
  // blocked right-hand sides: as many columns per launch as LDS and
  // residency allow
  int rmax = 1;
  for (int R = 2; R <= kMaxRhs; ++R) {
    CoopDev CR = C;
    CR.nrhs = R;
    const size_t l = coop_lds(CR);
    if (l > kLdsMax || coop_max_blocks(l) < nsub) break;
    rmax = R;
  }
  C.ld_t = (int)(((std::max(1, lv.nflat_g) * 8 + 255) / 256) * 32);
  C.ld_b = (int)(((std::max(1, lv.nflat_c) * 8 + 255) / 256) * 32);
  std::vector<int64_t> kioff(nsub + 1, 0), moff(nsub + 1, 0);
  int nmax_ops = 0;
  for (int s = 0; s < nsub; ++s) {
    const int64_t nI = T.n_int[s], ng = T.ngam(s);
    kioff[s + 1] = kioff[s] + nI * nI;
    moff[s + 1] = moff[s] + nI * ng;
    nmax_ops = std::max<int>(nmax_ops, (int)(nI * nI + nI * ng));
  }
  Arena& A = h->coop_arena;
  auto lay = [&] {
    C.Kinv = A.take<double>(std::max<int64_t>(1, kioff[nsub]));
    C.kioff = A.take<int64_t>(nsub + 1);
    C.Mt = A.take<double>(std::max<int64_t>(1, moff[nsub]));
    C.moff = A.take<int64_t>(nsub + 1);
    C.ops = A.take<double>((size_t)opoff[nsub]);
    C.opoff = A.take<int64_t>(nsub + 1);
    C.idx = A.take<int32_t>(idx.size());
    C.idxoff = A.take<int64_t>(nsub + 1);
    C.meta = A.take<int32_t>(meta.size());
    C.cg = A.take<int32_t>(cg.size());
    C.LLinv = A.take<double>((size_t)ncL * ncL);
    C.bar = A.take<unsigned>(2);
    C.sub_of_flat = A.take<int32_t>(sub_of_flat.size());
    C.t = A.take<double>((size_t)rmax * C.ld_t);
    C.da = A.take<double>((size_t)rmax * C.ld_t);
    C.b = A.take<double>((size_t)rmax * C.ld_b);
  };
  A.reset_sizing();
  lay();
  A.allocate(h->stream);
  lay();
  hipStream_t st = h->stream;
  Staging stg(st, &h->staged);
  stg.add(const_cast<int64_t*>(C.opoff), opoff);
  stg.add(const_cast<int32_t*>(C.idx), idx);
  stg.add(const_cast<int64_t*>(C.idxoff), idxoff);
  stg.add(const_cast<int32_t*>(C.meta), meta);
  stg.add(const_cast<int32_t*>(C.cg), cg);
  stg.add(const_cast<int32_t*>(C.sub_of_flat), sub_of_flat);
  stg.add(const_cast<int64_t*>(C.kioff), kioff);
  stg.add(const_cast<int64_t*>(C.moff), moff);
  stg.flush();
  BDDC_HIP(hipMemsetAsync(C.bar, 0, 2 * sizeof(unsigned), st));
  launch_wide_ops(st, lv.dev, nmax_ops, const_cast<double*>(C.Kinv), C.kioff, const_cast<double*>(C.Mt), C.moff);
  launch_pack_coop(st, lv.dev, C);
  launch_tri_inverse_dense(st, h->AL, ncL, ncL, const_cast<double*>(C.LLinv));
  C.b1 = l1.d.b;
  C.u2 = l1.d.uc;
  C.stop = nullptr;
  C.status = h->status;
  h->coop = C;
  h->coop_deep = true;
  h->coop_rmax = rmax;
  const char* cl = getenv("BDDC_COOP_LAUNCH");
  h->coop_launch = cl && std::string(cl) == "1";
  // operators and index lists once per workgroup, the level-1 contributions,
  // t / b / delta T g written and read back, the level-2 solution written
  h->coop_bytes = 8.0 * (double)opoff[nsub] + 4.0 * (double)idx.size() +
                  (double)nsub * (4.0 * cg.size() + 8.0 * ncL * ncL) + 8.0 * (double)lv.nflat_c * 2 +
                  8.0 * (double)lv.nflat_g * 4 + 8.0 * (double)l1.nflat_c + 8.0 * (double)lv.n;
  return true;
}

// One deep level whose substructures do not fit the cooperative kernel: dense
// K_II^-1 and M^T per level-2 substructure, applied in row blocks.
static bool plan_wide(bddc_ctx* h) {
  h->wide_deep = false;
  if (h->levels.size() != 2) return false;
  const char* env = getenv("BDDC_DEEP_PATH");
  if (env && std::string(env) != "wide") return false;
  Level& l1 = *h->levels[0];
  Level& lv = *h->levels[1];
  const Topology& T = lv.topo;
  const int nsub = lv.nsub;
  if (nsub < 1 || lv.nc < 1) return false;
  std::vector<int64_t> kioff(nsub + 1, 0), moff(nsub + 1, 0);
  int nmax_ops = 0;
  for (int s = 0; s < nsub; ++s) {
    const int64_t nI = T.n_int[s], ng = T.ngam(s);
    kioff[s + 1] = kioff[s] + nI * nI;
    moff[s + 1] = moff[s] + nI * ng;
    nmax_ops = std::max<int>(nmax_ops, (int)(nI * nI + nI * ng));
  }
  // the coarsest solve and the level-2 interface live in one workgroup's LDS
  if ((!h->coarse_inv && sizeof(double) * (size_t)lv.nc > kLdsLimit) ||
      sizeof(double) * ((size_t)lv.ngmax + kNT) > kLdsLimit ||
      sizeof(double) * (size_t)lv.nImax * kMaxRhs > kLdsMax)
    return false;
  std::vector<int32_t> sub_of_flat(lv.nflat_g);
  for (int s = 0; s < nsub; ++s)
    for (int f = lv.goff[s]; f < lv.goff[s + 1]; ++f) sub_of_flat[f] = s;
  WideDev W{};
  Arena& A = h->wide_arena;
  auto colpad = [](int64_t n) { return (int)(((std::max<int64_t>(n, 1) * 8 + 255) / 256) * 32); };
  const int ldi = colpad(lv.nflat_i), ldg = colpad(lv.nflat_g), ldc = colpad(lv.nflat_c), ldr = colpad(lv.n);
  double *cy = nullptr, *ct = nullptr, *ca = nullptr, *cv = nullptr, *cb = nullptr, *cr = nullptr, *ci = nullptr;
  auto lay = [&] {
    W.Kinv = A.take<double>(std::max<int64_t>(1, kioff[nsub]));
    W.kioff = A.take<int64_t>(nsub + 1);
    W.Mt = A.take<double>(std::max<int64_t>(1, moff[nsub]));
    W.moff = A.take<int64_t>(nsub + 1);
    W.sub_of_flat = A.take<int32_t>(std::max(1, lv.nflat_g));
    // level-2 scratch and r_2 for up to kMaxRhs columns
    cy = A.take<double>((size_t)kMaxRhs * ldi);
    ct = A.take<double>((size_t)kMaxRhs * ldg);
    ca = A.take<double>((size_t)kMaxRhs * ldg);
    cv = A.take<double>((size_t)kMaxRhs * ldg);
    cb = A.take<double>((size_t)kMaxRhs * ldc);
    cr = A.take<double>((size_t)kMaxRhs * ldr);
    ci = A.take<double>((size_t)kMaxRhs * ldi);
  };
  A.reset_sizing();
  lay();
  A.allocate(h->stream);
  lay();
  hipStream_t st = h->stream;
  {
    Staging stg(st, &h->staged);
    stg.add(const_cast<int64_t*>(W.kioff), kioff);
    stg.add(const_cast<int64_t*>(W.moff), moff);
    stg.add(const_cast<int32_t*>(W.sub_of_flat), sub_of_flat);
    stg.flush();
  }
  launch_wide_ops(st, lv.dev, nmax_ops, const_cast<double*>(W.Kinv), W.kioff, const_cast<double*>(W.Mt), W.moff);
  W.L = lv.dev;
  W.L.y = cy;
  W.L.t = ct;
  W.L.a = ca;
  W.L.v = cv;
  W.L.b = cb;
  W.ld_i = ldi;
  W.ld_g = ldg;
  W.ld_c = ldc;
  W.ld_r2 = ldr;
  W.rIf = ci;
  W.n2 = lv.n;
  W.nflat_i = lv.nflat_i;
  W.nImax = lv.nImax;
  W.ngmax = lv.ngmax;
  W.rows1 = 8;
  W.nchunk1 = std::max(1, (lv.nmax + W.rows1 - 1) / W.rows1);
  W.nchunk4 = std::max(1, (lv.nImax + 63) / 64);
  W.b1 = l1.d.b;
  W.csh_ptr1 = l1.d.csh_ptr;
  W.csh_flat1 = l1.d.csh_flat;
  W.r2 = cr;
  W.u2 = l1.d.uc;
  W.ncL = lv.nc;
  W.AL = h->AL;
  W.coarse_inv = h->coarse_inv ? 1 : 0;
  W.r3 = h->coarse_r;
  W.u3 = h->coarse_u;
  W.ld_3 = h->ld_cr;
  W.nflat = lv.nflat_g;
  h->wide = W;
  h->wide_deep = true;
  // K_II^-1, M^T twice, T_rr, Psi twice, and the level vectors
  double by = 0, op_pre = 0, op_res = 0, op_crs = 0, op_post = 0;
  for (int s = 0; s < nsub; ++s) {
    const double nI = T.n_int[s], ng = T.ngam(s), nr = T.n_r[s], ncs = lv.coff[s + 1] - lv.coff[s];
    by += 8 * (nI * nI + 2 * nI * ng + nr * nr + 2 * ng * ncs);
    op_pre += 8 * (nI * nI + nI * ng);
    op_res += 8 * (nr * nr + ng * ncs);
    op_crs += 8 * (ng * ncs);
    op_post += 8 * (nI * ng);
  }
  h->wide_bytes = by + 8.0 * (2.0 * l1.nflat_c + 3.0 * lv.n + 6.0 * lv.nflat_g + lv.nflat_c + lv.nc);
  // per launch: the gather of r_2 and y, t written; g, delta T g, b; u_3 and
  // v; u_B and y read, u_I and u_2 written
  h->wide_by[0] = op_pre + 8.0 * (2.0 * l1.nflat_c + lv.n + lv.nflat_i + lv.nflat_g);
  h->wide_by[1] = op_res + 8.0 * (3.0 * lv.nflat_g + lv.nflat_c);
  h->wide_by[2] = op_crs + 8.0 * (lv.nflat_c + 2.0 * lv.nc + 2.0 * lv.nflat_g);
  h->wide_by[3] = op_post + 8.0 * (2.0 * lv.nflat_i + 2.0 * lv.nflat_g + lv.n);
  return true;
}

// decide whether the deep levels fit one workgroup and fill the fused-kernel arguments
static void plan_deep(bddc_ctx* h) {
  h->fused_deep = false;
  const int L = (int)h->levels.size();
  h->deep_sel = BDDC_DEEP_LEVELS;
  if (L < 2 || L - 1 > kMaxDeep) return;
  // one deep level: both the cooperative and the row-block path where they
  // apply (the tuning chooses; the cooperative one first)
  const bool coop = plan_coop(h);
  const bool wide = plan_wide(h);
  if (coop || wide) {
    h->deep_sel = coop ? BDDC_DEEP_COOP : BDDC_DEEP_WIDE;
    return;
  }
  const char* env = getenv("BDDC_DEEP_PATH");
  if (env && (std::string(env) == "levels" || std::string(env) == "coop" || std::string(env) == "wide")) return;
  double bytes = 0;
  int wstride = 1;
  for (int li = 1; li < L; ++li) {
    const Level& lv = *h->levels[li];
    const Topology& T = lv.topo;
    for (int s = 0; s < lv.nsub; ++s) {
      const double nI = T.n_int[s], ng = T.ngam(s), nr = T.n_r[s], ncs = lv.coff[s + 1] - lv.coff[s];
      bytes += 8 * (nI * nI + ng * nI + nr * nr + 2 * ng * ncs);
    }
    wstride = std::max({wstride, 2 * lv.nImax, lv.ngmax + lv.nImax, lv.ncsmax, lv.ngmax});
  }
  const int ncL = h->levels.back()->nc;
  if (h->coarse_inv) return;   // the fused kernel solves the coarsest problem with its Cholesky factor
  const bool forced = env && std::string(env) == "fused";
  if (!forced && bytes > 4.0e6) return;
  if (deep_lds(wstride, ncL) > kLdsLimit) return;
  DeepArgs& A = h->deep;
  A = DeepArgs{};
  A.nlev = L - 1;
  for (int dl = 0; dl < A.nlev; ++dl) {
    Level& lv = *h->levels[dl + 1];
    Level& up = *h->levels[dl];
    A.lv[dl] = lv.dev;
    A.lv[dl].stop = nullptr;
    A.rvec[dl] = up.d.rc;
    A.uvec[dl] = up.d.uc;
    A.nvec[dl] = up.nc;
  }
  A.rc_last = h->levels.back()->d.rc;
  A.uc_last = h->levels.back()->d.uc;
  A.ncL = ncL;
  A.LL = h->AL;
  Level& l1 = *h->levels[0];
  A.n2 = l1.nc;
  A.csh_ptr1 = l1.d.csh_ptr;
  A.csh_flat1 = l1.d.csh_flat;
  A.b1 = l1.d.b;
  A.wstride = wstride;
  h->fused_deep = true;
  h->deep_sel = BDDC_DEEP_FUSED;
}

// symmetric tridiagonal extreme eigenvalues by Sturm bisection
static double tri_eig(const std::vector<double>& a, const std::vector<double>& b, bool largest) {
  const int n = (int)a.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0) + (i + 1 < n ? std::fabs(b[i]) : 0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {
    int c = 0;
    double q = 1.0;
    for (int i = 0; i < n; ++i) {
      q = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q < 0) ++c;
    }
    return c;
  };
  const int target = largest ? n - 1 : 0;   // index of the eigenvalue
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) > target) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

static double lanczos_kappa(const std::vector<double>& al, const std::vector<double>& be) {
  const int k = (int)al.size();
  if (k == 0) return 1.0;
  std::vector<double> a(k), b(std::max(0, k - 1));
  for (int i = 0; i < k; ++i) {
    a[i] = 1.0 / al[i] + (i > 0 ? be[i - 1] / al[i - 1] : 0.0);
    if (i + 1 < k) b[i] = std::sqrt(std::max(0.0, be[i])) / al[i];
  }
  const double mx = tri_eig(a, b, true), mn = tri_eig(a, b, false);
  return mn > 0 ? mx / mn : 0.0;
}

// One chunk of PCG launches as a HIP graph, captured on first use and kept by
// the handle (its launches have fixed arguments).  Not while kernel timing is
// armed (its events cannot be captured), nor with BDDC_PCG_GRAPH=0; returns
// false when the chunk must be launched directly.
template <class F>
static bool graph_chunk(bddc_ctx* h, hipStream_t st, F&& enqueue) {
  if (h->graph_off || h->noalloc_now || timing::active()) return false;
  // cooperative launches are issued directly, not replayed from a graph
  if (h->coop_shared && h->deep_sel == BDDC_DEEP_COOP) return false;
  if (!h->graph_exec) {
    const char* env = getenv("BDDC_PCG_GRAPH");
    if (env && std::string(env) == "0") {
      h->graph_off = true;
      return false;
    }
    // captured on a stream of the library's own (the caller's may be the
    // null stream, which cannot be captured); replayed on the caller's.
    // Relaxed mode: other threads' synchronising calls stay legal meanwhile
    // (the capture itself only enqueues kernels)
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess ||
        hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
      (void)hipGetLastError();
      if (cs) (void)hipStreamDestroy(cs);
      h->graph_off = true;
      return false;
    }
    hipGraph_t g = nullptr;
    try {
      enqueue(cs);
    } catch (...) {
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      (void)hipStreamDestroy(cs);
      (void)hipGetLastError();
      throw;
    }
    const hipError_t e1 = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    hipGraphExec_t ex = nullptr;
    const hipError_t e2 = (e1 == hipSuccess && g) ? hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) : e1;
    size_t nodes = 0;
    if (g) (void)hipGraphGetNodes(g, nullptr, &nodes);
    if (g) (void)hipGraphDestroy(g);
    if (getenv("BDDC_HOST_TIMING"))
      fprintf(stderr, "libbddc pcg graph: %s (%zu nodes)\n", e2 == hipSuccess ? "captured" : hipGetErrorString(e2),
              nodes);
    if (e2 != hipSuccess || !ex) {
      (void)hipGetLastError();
      h->graph_off = true;
      return false;
    }
    h->graph_exec = ex;
  }
  BDDC_HIP(hipGraphLaunch(h->graph_exec, st));
  return true;
}

// The per-column PCG state for R columns, laid out in A (a sizing pass when A
// holds no memory yet).
static void lay_columns(bddc_ctx* h, Arena& A, int R) {
  Level& l1 = *h->levels[0];
  PcgDev& P = h->pcg;
  auto pad = [](int64_t n) { return (int)(((std::max<int64_t>(n, 1) * 8 + 255) / 256) * 32); };   // 256-byte columns
  P.ld_if = pad(P.nif);
  P.ld_flat = pad(l1.nflat_g);
  P.ld_cflat = pad(l1.nflat_c);
  P.ld_coarse = pad(l1.nc);
  P.ld_sub = pad(std::max(P.nsub1, P.npq));
  P.ld_blk = pad(P.nblk);
  h->ld_cy = pad(l1.nflat_i);
  P.x = A.take<double>((size_t)R * P.ld_if);
  P.r[0] = A.take<double>((size_t)R * P.ld_if);
  P.r[1] = A.take<double>((size_t)R * P.ld_if);
  P.p[0] = A.take<double>((size_t)R * P.ld_if);
  P.p[1] = A.take<double>((size_t)R * P.ld_if);
  P.z = A.take<double>((size_t)R * P.ld_if);
  P.pq_part = A.take<double>((size_t)R * P.ld_sub);
  P.rr_part = A.take<double>((size_t)R * P.ld_sub);
  P.rz_part[0] = A.take<double>((size_t)R * P.ld_blk);
  P.rz_part[1] = A.take<double>((size_t)R * P.ld_blk);
  P.qloc = A.take<double>((size_t)R * P.ld_flat);
  P.da = A.take<double>((size_t)R * P.ld_flat);
  P.gflat = A.take<double>(P.nrb ? (size_t)R * P.ld_flat : 0);
  P.b = A.take<double>((size_t)R * P.ld_cflat);
  P.uc = A.take<double>((size_t)R * P.ld_coarse);
  P.sc = A.take<PcgScalars>(R);
  P.tail_cnt = A.take<unsigned int>(3 * kTailStride);
  P.slot_cnt = A.take<unsigned int>(2 * kSlots * 16);
  P.slotv = A.take<double>(3 * kSlots);
  h->cy = A.take<double>((size_t)R * h->ld_cy);
  h->ct = A.take<double>((size_t)R * P.ld_flat);
}

// The per-column PCG state for R columns (reallocated when a solve needs more
// columns than the arena holds; a captured chunk keeps the old addresses, so
// it is dropped).
static void ensure_columns(bddc_ctx* h, int R) {
  if (h->cols_cap >= R) return;
  if (h->noalloc_now) fail(BDDC_EUNSUPPORTED, "the no-allocation solve needs more columns than it laid out");
  BDDC_HIP(hipStreamSynchronize(h->stream));
  h->cols_arena.release(h->stream);
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  h->graph_exec = nullptr;
  h->graph_nrhs = 0;
  Arena& A = h->cols_arena;
  A.reset_sizing();
  lay_columns(h, A, R);
  A.allocate(h->stream);
  lay_columns(h, A, R);
  h->cols_cap = R;
}

// PCG on the level-1 interface for R <= kMaxRhs right-hand sides at once
// (columns of f and u at stride ld), in three parts so that a caller can
// interleave several solves: pcg_begin enqueues the condensation, r_0 and
// z_0; pcg_advance enqueues chunks of iterations and an asynchronous copy of
// the convergence flags; pcg_finish waits, recovers the interior and reports.
// Each column runs its own recurrences and convergence test; the launches of
// one iteration serve every column still iterating.

// Iteration k: matvec, update + restriction, deep levels, prolongation with
// the convergence test, post.  The test sits in the prolongation, so at the
// converged iteration K the update, restriction and deep levels still run
// (tagged k - 1: they work iff k <= K) and the rest return at once.  The
// kernels take their iteration as sc[0].it_base + u (u < 0: iteration 0), so
// one chunk of launches is the same for every chunk and can be replayed as a
// HIP graph.
// whether the sums of the PCG partials take launches of their own (p^T S p
// and r.z; r.r: rr_sum_needed)
static bool sum_launches(const PcgDev& P) { return P.fin == 1 || (P.fin >= 2 && P.nrhs > 1); }
static bool rr_sum_needed(const PcgDev& P) { return sum_launches(P) || P.fin == 3; }

// BDDC_RR_SUM=launch keeps the r.r sum in a launch of its own on the wide path
static bool rr_sum_launch() {
  const char* e = getenv("BDDC_RR_SUM");
  return e && std::string(e) == "launch";
}

static void pcg_apply_iface(bddc_ctx* h, hipStream_t q, int uu, int it) {
  Level& l1 = *h->levels[0];
  PcgDev& P = h->pcg;
  timing::current_tag = it - 1;
  if (P.nrb) {
    // wide interfaces: the update once per substructure, then the
    // restriction by row blocks
    if (it > 0) launch_pcg_update_rows(q, l1.dev, P, uu);
    timing::Scope ts("apply_restrict", h->by_r_prec, 0);
    launch_pcg_restrict_rows(q, l1.dev, l1.ngmax, P, uu);
  } else {
    timing::Scope ts("apply_restrict", it > 0 ? h->by_ur_prec : h->by_r_prec, 0);
    launch_pcg_update_restrict(q, l1.dev, l1.ngmax, l1.nrmax, l1.ncsmax, P, uu);
  }
  // r.r is read by the convergence test of the prolongation: the deep
  // launches may sum it (the wide path), else a launch of its own does
  const bool want_rr = rr_sum_needed(P) && it > 0;
  const bool rr_done = run_deep_cols(h, q, P.b, P.ld_cflat, const_cast<double*>(P.uc), P.ld_coarse, P.nrhs,
                                     want_rr && !rr_sum_launch() ? &P : nullptr);
  if (want_rr && !rr_done) launch_pcg_sum(q, P, 1, uu);
  timing::current_tag = it;
  {
    timing::Scope ts("apply_average", h->by_average, 0);
    launch_pcg_prolong_post(q, l1.dev, P, uu);
  }
  if (sum_launches(P)) launch_pcg_sum(q, P, 2, uu);
}

static void pcg_chunk(bddc_ctx* h, hipStream_t q, int it0) {
  Level& l1 = *h->levels[0];
  PcgDev& P = h->pcg;
  for (int uu = 0; uu < h->pcg_check; ++uu) {
    const int it = it0 + uu;
    timing::current_tag = it;
    {
      // the product of iteration k works iff k <= K (K = converged iteration)
      timing::Scope ts("schur_local", h->by_schur_packed, 0, -1);
      if (P.nrb)
        launch_pcg_matvec_rows(q, l1.dev, l1.ngmax, P, uu);
      else
        launch_pcg_matvec(q, l1.dev, l1.ngmax, P, uu);
    }
    if (sum_launches(P)) launch_pcg_sum(q, P, 0, uu);
    pcg_apply_iface(h, q, uu, it);
  }
  launch_pcg_advance(q, P, h->pcg_check);
}

static void pcg_begin(bddc_ctx* h, const double* f, int64_t ld, int R, double rtol, int maxit) {
  hipStream_t st = h->stream;
  Level& l1 = *h->levels[0];
  ensure_columns(h, R);
  PcgDev& P = h->pcg;
  P.nrhs = R;
  PcgRun& run = h->run;
  run = PcgRun{};
  run.f = f;
  run.ld = ld;
  run.R = R;
  run.maxit = maxit;
  if (h->coop_deep) {
    h->coop_shared = g_live_handles.load() > 1;
    launch_coop_reset(st, h->coop);
  }
  if (P.fin == 2 && R == 1) launch_tail_reset(st, P);
  if (P.fin == 3 && R == 1) launch_slot_reset(st, P);
  const int nif = (int)l1.iface_dof.size();
  const int nb = h->nblk;
  const int nbf = std::min(1024, std::max(1, (int)((h->n_free + kNT - 1) / kNT)));
  PcgScalars* sch = h->sc_host;
  for (int c = 0; c < R; ++c) {
    std::memset(&sch[c], 0, offsetof(PcgScalars, alphas));
    sch[c].maxit = maxit;
    sch[c].rtol2 = rtol * rtol;   // thr2 = rtol^2 ||f||^2 is formed on the device
    sch[c].it_base = 1;
    BDDC_HIP(hipMemcpyAsync(P.sc + c, sch + c, offsetof(PcgScalars, alphas), hipMemcpyHostToDevice, st));
  }
  // the condensation: with the tiled block substitution (the level-1 factor
  // of the tiled elimination; BDDC_IR_PATH=sweep: not taken) or the streamed
  // sweeps all columns in one pass over L (y = L^{-1} f_I, t = L_GI y per
  // column); else the blocked triangular solves when kMaxRhs columns fit the
  // LDS, else column by column
  {
    const char* ir = getenv("BDDC_IR_PATH");
    run.tiles = l1.big && !(ir && std::string(ir) == "sweep");
  }
  run.sweep = !run.tiles && use_sweep(l1.nmax);
  run.blocked = !run.sweep && !run.tiles && apply_cols_lds(kMaxRhs, l1.nImax, l1.ngmax) <= kLdsMax;
  const bool sweep = run.sweep, tiles = run.tiles, blocked = run.blocked;
  if (sweep) launch_sweep_pre_cols(st, l1.dev, f, ld, h->cy, h->ld_cy, h->ct, P.ld_flat, R);
  if (tiles) launch_tile_pre_cols(st, l1.dev, f, ld, h->cy, h->ld_cy, h->ct, P.ld_flat, R);
  if (blocked) launch_apply_pre_cols(st, l1.dev, l1.nImax, l1.ngmax, f, ld, h->cy, h->ld_cy, h->ct, P.ld_flat, R);
  for (int c = 0; c < R; ++c) {
    const double* fc = f + (size_t)c * ld;
    double* rc = P.r[0] + (size_t)c * P.ld_if;
    launch_dot_partial(st, nbf, (int)h->n_free, fc, fc, h->partial);
    launch_scalar(st, 4, nbf, h->partial, P.sc + c);                 // bb, thr2 = rtol^2 bb
    if (!sweep && !tiles && !blocked) launch_apply_pre(st, l1.dev, l1.nImax, l1.ngmax, fc);
    const double* tc = sweep || tiles || blocked ? h->ct + (size_t)c * P.ld_flat : l1.d.t;
    launch_condense(st, nif, l1.d.sh_ptr, l1.d.sh_flat, l1.d.iface_dof, fc, tc, rc, P.x + (size_t)c * P.ld_if);
    launch_dot_partial(st, nb, nif, rc, rc, h->partial);
    launch_scalar(st, 5, nb, h->partial, P.sc + c);                  // rr0, done if already small
  }
  // every kernel below returns at once once every column has finished
  for (auto& lvp : h->levels) lvp->dev.stop = &P.sc[0].all_done;
  run.tmark = timing::mark();
  // z_0 = M r_0 and its r.z partials (parity 0)
  pcg_apply_iface(h, st, -1, 0);
  if (h->graph_exec && h->graph_nrhs != R && !h->noalloc_now) {
    (void)hipGraphExecDestroy(h->graph_exec);
    h->graph_exec = nullptr;
  }
  run.active = true;
}

// Enqueue chunks covering at least `iters` more iterations (iterations past
// maxit or convergence return at once), then an asynchronous copy of the
// convergence flags to the pinned host scalars and an event after it.
static void pcg_advance(bddc_ctx* h, int iters) {
  hipStream_t st = h->stream;
  PcgRun& run = h->run;
  const int R = run.R;
  for (int done = 0; done < std::max(1, iters) && run.it < run.maxit; done += h->pcg_check) {
    if (graph_chunk(h, st, [&](hipStream_t q) { pcg_chunk(h, q, run.it + 1); }))
      h->graph_nrhs = R;
    else
      pcg_chunk(h, st, run.it + 1);
    run.it += h->pcg_check;
  }
  timing::current_tag = -1;
  BDDC_HIP(hipMemcpyAsync(h->sc_host, h->pcg.sc, offsetof(PcgScalars, alphas), hipMemcpyDeviceToHost, st));
  if (!h->run_event) BDDC_HIP(hipEventCreateWithFlags(&h->run_event, hipEventDisableTiming));
  BDDC_HIP(hipEventRecord(h->run_event, st));
}

// 1 when the iterations enqueued so far have finished every column (or
// reached maxit), 0 when more are needed, -1 while the last advance runs.
static int pcg_poll(bddc_ctx* h, bool wait) {
  PcgRun& run = h->run;
  if (wait) {
    BDDC_HIP(hipEventSynchronize(h->run_event));
  } else {
    const hipError_t e = hipEventQuery(h->run_event);
    if (e == hipErrorNotReady) return -1;
    BDDC_HIP(e);
  }
  return (h->sc_host[0].all_done || run.it >= run.maxit) ? 1 : 0;
}

// Interior recovery and the per-column results; synchronises the stream.
// Returns the number of columns that did not converge.
static int pcg_finish(bddc_ctx* h, double* u, int64_t ld, int32_t* iters_out, double* relres) {
  hipStream_t st = h->stream;
  Level& l1 = *h->levels[0];
  PcgDev& P = h->pcg;
  PcgRun& run = h->run;
  const int R = run.R;
  const double* f = run.f;
  struct Clear {
    bddc_ctx* h;
    ~Clear() {
      for (auto& lvp : h->levels) lvp->dev.stop = nullptr;
      timing::current_tag = -1;
      h->run.active = false;
    }
  } clear{h};
  timing::current_tag = -1;
  // interior recovery u_I = L^-T (y - L_GI^T x) with each column's own y:
  // the column sweeps, the tiled and the blocked solves kept every column's
  // y; column by column, the set-up pass left the last column's y (the
  // level's stop flag is raised by now, so these launches go without it)
  LevelDev L1 = l1.dev;
  L1.stop = nullptr;
  if (run.sweep) {
    launch_sweep_recover_cols(st, L1, P.x, P.ld_if, h->cy, h->ld_cy, u, ld, R);
  } else if (run.tiles) {
    launch_tile_recover_cols(st, L1, P.x, P.ld_if, h->cy, h->ld_cy, u, ld, R, l1.ngmax);
  } else if (run.blocked) {
    launch_recover_cols(st, L1, l1.nImax, l1.ngmax, P.x, P.ld_if, h->cy, h->ld_cy, u, ld, R);
  } else {
    for (int c = R - 1; c >= 0; --c) {
      if (c < R - 1) launch_apply_pre(st, L1, l1.nImax, l1.ngmax, f + (size_t)c * run.ld);
      launch_recover(st, L1, l1.nImax, l1.ngmax, P.x + (size_t)c * P.ld_if, u + (size_t)c * ld);
    }
  }
  PcgScalars* sch = h->sc_host;
  int dev_status = 0;
  for (int c = 0; c < R; ++c) BDDC_HIP(hipMemcpyAsync(sch + c, P.sc + c, sizeof(PcgScalars), hipMemcpyDeviceToHost, st));
  BDDC_HIP(hipMemcpyAsync(&dev_status, h->status, sizeof(int), hipMemcpyDeviceToHost, st));
  BDDC_HIP(hipStreamSynchronize(st));
  if (dev_status & 4) fail(BDDC_EDEVICE, "a grid barrier of the deep-level kernel timed out");
  int maxiters = 0, failed = 0;
  for (int c = 0; c < R; ++c) {
    const PcgScalars& S = sch[c];
    iters_out[c] = S.iters;
    relres[c] = S.bb > 0 ? std::sqrt(S.rr / S.bb) : 0.0;
    if (S.done != 1) ++failed;
    maxiters = std::max(maxiters, S.iters);
  }
  // launches of iteration k work iff k < K (the product: k <= K, tagged k-1)
  timing::prune(run.tmark, maxiters);
  const PcgScalars& S = sch[R - 1];
  std::vector<double> al(S.alphas, S.alphas + std::min(S.iters, kMaxHist));
  std::vector<double> be(S.betas, S.betas + std::max(0, std::min(S.iters, kMaxHist) - 1));
  h->info.kappa = lanczos_kappa(al, be);
  h->info.last_iters = S.iters;
  return failed;
}

// The blocking solve: begin, chunks until every column has finished, finish.
static int pcg_block(bddc_ctx* h, const double* f, double* u, int64_t ld, int R, double rtol, int maxit,
                     int32_t* iters_out, double* relres) {
  struct Abort {
    bddc_ctx* h;
    ~Abort() {
      if (h->run.active) {
        for (auto& lvp : h->levels) lvp->dev.stop = nullptr;
        timing::current_tag = -1;
        h->run.active = false;
      }
    }
  } abort_guard{h};
  pcg_begin(h, f, ld, R, rtol, maxit);
  while (h->run.it < maxit) {
    pcg_advance(h, h->pcg_check);
    if (pcg_poll(h, true) == 1) break;
  }
  return pcg_finish(h, u, ld, iters_out, relres);
}

static int64_t model_bytes(const bddc_ctx* h, bool apply) {
  // algorithmic bytes of one interface operator product / one preconditioner apply
  int64_t bytes = 0;
  for (size_t li = 0; li < h->levels.size(); ++li) {
    const Level& lv = *h->levels[li];
    const Topology& T = lv.topo;
    for (int s = 0; s < lv.nsub; ++s) {
      const int64_t nI = T.n_int[s], ng = T.ngam(s), nr = T.n_r[s];
      const int64_t ncs = lv.coff[s + 1] - lv.coff[s];
      if (!apply) {
        if (li == 0) bytes += 8 * ng * ng;
        continue;
      }
      bytes += 8 * (nr * nr + 2 * ng * ncs);                       // T_rr once, Psi twice
      if (li > 0) bytes += 8 * (nI * (nI + 1) + 2 * ng * nI);      // L_II two sweeps (lower), L_GI twice
    }
    if (!apply) {
      if (li == 0) bytes += 8 * (int64_t)(3 * lv.nflat_g + 3 * lv.iface_dof.size());
      break;
    }
    bytes += 8 * (int64_t)(6 * lv.nflat_g + 3 * lv.nflat_c + 2 * lv.iface_dof.size() + 2 * lv.nc);
  }
  if (apply) bytes += 8 * (int64_t)h->ncL * (h->ncL + 1);
  return bytes;
}

}  // namespace bddc

// ===========================================================================
using namespace bddc;

namespace {

thread_local std::string g_last_error;

bddc_status guard(const std::function<void()>& fn) {
  try {
    fn();
    return BDDC_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    if (getenv("BDDC_VERBOSE")) fprintf(stderr, "libbddc: %s\n", e.msg.c_str());
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return BDDC_ENOMEM;
  } catch (...) {
    g_last_error = "unexpected exception";
    return BDDC_EDEVICE;
  }
}

void release(bddc_ctx* h) {
  if (!h) return;
  if (h->counted) g_live_handles.fetch_sub(1);
  hipStream_t st = h->stream;
  (void)hipStreamSynchronize(st);
  for (auto& lv : h->levels) {
    lv->arena_a.release(st);
    lv->arena_b.release(st);
    lv->arena_pcg.release(st);
  }
  h->top.release(st);
  h->coop_arena.release(st);
  h->wide_arena.release(st);
  h->cols_arena.release(st);
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  h->graph_exec = nullptr;
  if (h->run_event) (void)hipEventDestroy(h->run_event);
  pinned_release(h->sc_host);
  for (void* b : h->staged) pinned_release(b);
  delete h;   // the pool frees above are stream-ordered
}

void fill_level_info(const Level& lv, int idx, bddc_info* info) {
  info->nsub[idx] = lv.nsub;
  info->n_dof[idx] = lv.n;
  info->n_interface[idx] = (int32_t)lv.iface_dof.size();
  info->n_corners[idx] = (int32_t)lv.topo.corners.size();
  info->n_edges[idx] = lv.nedge;
  info->nc[idx] = lv.nc;
  info->n_adaptive[idx] = lv.n_adaptive;
  info->omega[idx] = lv.omega;
}

}  // namespace

extern "C" {

const char* bddc_last_error(void) { return g_last_error.c_str(); }

const char* bddc_status_string(bddc_status s) {
  switch (s) {
    case BDDC_OK: return "ok";
    case BDDC_EINVAL: return "invalid argument";
    case BDDC_ENOMEM: return "out of device memory";
    case BDDC_ESINGULAR: return "singular local or coarse problem";
    case BDDC_EPARTITION: return "invalid partition";
    case BDDC_ENOCONV: return "PCG did not converge within maxit";
    case BDDC_EDEVICE: return "HIP runtime error";
    case BDDC_EBUSY: return "busy";
    case BDDC_EUNSUPPORTED: return "unsupported by this build";
  }
  return "unknown status";
}

bddc_status bddc_plan(const bddc_problem* p, bddc_info* info) {
  return guard([&] {
    HostClock clk;
    validate(p);
    clk.lap("validate");
    if (!info) fail(BDDC_EINVAL, "info is NULL");
    Level lv;
    const char* how = getenv("BDDC_CLASSIFY");
    if (how && std::string(how) == "elements") {
      // the general element-list classification (the one levels >= 2 use)
      Level1Elements E = level1_elements(p);
      lv.topo = classify((p->nx - 1) * (p->ny - 1), p->nsub, E.ptr, E.dof, E.sub, E.touch);
    } else {
      lv.topo = classify_grid(p->nx, p->ny, p->part, p->nsub, nullptr);
    }
    expand_node_topology(lv.topo, nullptr, dofs_per_node(p->element));
    clk.lap("classify");
    layout_level(lv);
    clk.lap("layout");
    std::memset(info, 0, sizeof(*info));
    info->n_free = (int64_t)dofs_per_node(p->element) * (p->nx - 1) * (p->ny - 1);
    info->levels = p->levels;
    fill_level_info(lv, 0, info);
    // device bytes a set-up will hold, from the level-1 sizes: the dense local
    // matrices (and the tiled kernel's diagonal inverses), the PCG operators
    // S_s and T_rr (full; packed is smaller), the level's flat arrays and one
    // column of PCG state; the deeper levels are a fraction of level 1 and
    // are covered by a 10% margin
    const Topology& T = lv.topo;
    double by = 0;
    for (int s = 0; s < lv.nsub; ++s) {
      const double n = T.nloc(s), ng = T.ngam(s), nI = T.n_int[s];
      by += 8.0 * n * n + 16.0 * ng * ng + 8.0 * ng * 8;
      if (level_big_chol(1, lv.nmax)) by += 8.0 * 64.0 * 64.0 * std::ceil(nI / 64.0);
    }
    by += 8.0 * (12.0 * lv.nflat_g + 4.0 * lv.nflat_i) + 8.0 * 10.0 * (double)info->n_free;
    info->device_bytes = (int64_t)(1.1 * by);
  });
}

}  // extern "C"

namespace bddc {
namespace {

// launch configurations chosen by the autotuner, by problem shape
std::mutex g_tune_mu;
std::map<std::string, bddc_tuning> g_tune_cache;

int deep_available(const bddc_ctx* h) {
  int m = 1 << BDDC_DEEP_LEVELS;
  if (h->coop_deep) m |= 1 << BDDC_DEEP_COOP;
  if (h->wide_deep) m |= 1 << BDDC_DEEP_WIDE;
  if (h->fused_deep) m |= 1 << BDDC_DEEP_FUSED;
  return m;
}

bddc_tuning current_tuning(const bddc_ctx* h) {
  bddc_tuning t{};
  t.deep_path = h->deep_sel;
  t.finalize = h->pcg.fin;
  t.graph = h->graph_off ? 0 : 1;
  t.check = h->pcg_check;
  t.available = deep_available(h);
  t.solve_ms = h->tuned_ms;
  return t;
}

void check_tuning(const bddc_ctx* h, const bddc_tuning& t) {
  if (t.deep_path < 0 || t.deep_path > BDDC_DEEP_LEVELS || !(deep_available(h) >> t.deep_path & 1))
    fail(BDDC_EINVAL, "deep path not available for this set-up");
  if (t.finalize < 0 || t.finalize > 3) fail(BDDC_EINVAL, "finalize must be 0, 1, 2 or 3");
  if (h->pcg.nrb && t.finalize != 1)
    fail(BDDC_EINVAL, "the row-block launches of wide interfaces take finalize 1 only");
  if (t.graph != 0 && t.graph != 1) fail(BDDC_EINVAL, "graph must be 0 or 1");
  if (t.check != 4 && t.check != 8 && t.check != 16) fail(BDDC_EINVAL, "check must be 4, 8 or 16");
}

// install a configuration; a captured chunk of launches no longer matches it
void apply_tuning(bddc_ctx* h, const bddc_tuning& t) {
  if (h->graph_exec) {
    BDDC_HIP(hipStreamSynchronize(h->stream));
    (void)hipGraphExecDestroy(h->graph_exec);
    h->graph_exec = nullptr;
    h->graph_nrhs = 0;
  }
  h->deep_sel = t.deep_path;
  h->pcg.fin = t.finalize;
  h->graph_off = t.graph == 0;
  h->pcg_check = t.check;
}

std::string shape_key(const bddc_ctx* h) {
  std::string k = std::to_string(h->nx) + "x" + std::to_string(h->ny) + " e" + std::to_string(h->element) + " c" +
                  std::to_string(h->constraints) + " p" + std::to_string(h->precision);
  for (const auto& lv : h->levels) k += " " + std::to_string(lv->nsub) + ":" + std::to_string(lv->nc);
  return k;
}

}  // namespace
}  // namespace bddc
extern "C" {

bddc_status bddc_setup(const bddc_problem* p, void* hip_stream, bddc_handle* out) {
  if (out) *out = nullptr;
  bddc_ctx* h = nullptr;
  bddc_status st = guard([&] {
    validate(p);
    if (!out) fail(BDDC_EINVAL, "out is NULL");
    h = new bddc_ctx();
    h->nx = p->nx;
    h->ny = p->ny;
    h->L = p->levels;
    h->element = p->element;
    h->constraints = p->constraints;
    h->precision = p->precision;
    h->tau = p->tau;
    h->n_free = (int64_t)dofs_per_node(p->element) * (p->nx - 1) * (p->ny - 1);
    h->nz = p->element == BDDC_Q1_ELASTIC ? 3 : 1;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    BDDC_HIP(hipGetDevice(&h->device));
    HostClock clk;
    Builder(h, p).run();
    clk.lap("builder");
    // PCG state on the level-1 interface
    Level& l1 = *h->levels[0];
    const int nif = (int)l1.iface_dof.size();
    h->nblk = std::min(256, std::max(1, (nif + kNT - 1) / kNT));
    Arena& B = h->levels[0]->arena_pcg;
    PcgDev& P = h->pcg;
    // per interface dof: the sharers' rows of the delta-weighted coarse basis
    // (row offsets here; the device fills the coarse ids and weights)
    std::vector<int32_t> sub_of_flat(l1.nflat_g), phi_ptr(nif + 1, 0);
    for (int s = 0; s < l1.nsub; ++s)
      for (int f = l1.goff[s]; f < l1.goff[s + 1]; ++f) sub_of_flat[f] = s;
    for (int gi = 0; gi < nif; ++gi) {
      int len = 0;
      for (int q = l1.sh_ptr[gi]; q < l1.sh_ptr[gi + 1]; ++q) {
        const int t = sub_of_flat[l1.sh_flat[q]];
        len += l1.coff[t + 1] - l1.coff[t];
      }
      phi_ptr[gi + 1] = phi_ptr[gi] + len;
    }
    const size_t nphi = (size_t)phi_ptr[nif];
    // packed lower triangles of S_s and T_rr
    // (interfaces wider than 64 dofs: full matrices, so that the rows a
    // workgroup reads are adjacent in memory for every column; their partial
    // row sums no longer fit the registers of the packed form)
    const char* oenv = getenv("BDDC_PCG_OPS");
    P.full = oenv ? std::string(oenv) == "full" : l1.ngmax > 64;
    {
      // interfaces wider than a workgroup: the product and the
      // update/restriction by 64-row blocks (full storage, one-block sums);
      // BDDC_PCG_ROWS=1/0 forces either (not the factored BF16 form)
      const char* renv = getenv("BDDC_PCG_ROWS");
      const bool rows = h->precision != BDDC_BF16 && (renv ? std::string(renv) == "1" : l1.ngmax > kNT);
      P.nrb = rows ? pcg_rows_blocks(l1.ngmax) : 0;
      P.fullpad = rows ? 1 : 0;
      if (rows) P.full = 1;
      if (h->precision == BDDC_BF16) {
        // the factored form stages W of a whole substructure in LDS
        const size_t nr = (size_t)l1.nrmax;
        const size_t lds = sizeof(double) * (3 * (size_t)l1.ngmax + kNT + nr + nr * (nr + 1) / 2) +
                           sizeof(float) * (nr * (size_t)l1.ncsmax + nr);
        if (lds > kLdsMax)
          fail(BDDC_EUNSUPPORTED, "the BF16 form needs the factored T_rr of each substructure in LDS; the widest "
                                  "interface is too large for it");
      }
    }
    std::vector<int64_t> spoff(l1.nsub + 1, 0), tpoff(l1.nsub + 1, 0);
    for (int s = 0; s < l1.nsub; ++s) {
      const int64_t ng = l1.topo.ngam(s), nr = l1.topo.n_r[s];
      const int64_t lds_ = P.fullpad ? pad_ld((int)ng, 8) : ng;
      const int64_t ldt = P.fullpad ? pad_ld((int)nr, h->precision == BDDC_FP32 ? 4 : 8) : nr;
      spoff[s + 1] = spoff[s] + (P.full ? lds_ * ng : ng * (ng + 1) / 2);
      tpoff[s + 1] = tpoff[s] + (P.full ? ldt * nr : nr * (nr + 1) / 2);
    }
    // every sharer's flat entry of each flat entry's dof, padded to four
    bool fits4 = true;
    for (int gi = 0; gi < nif; ++gi) fits4 = fits4 && l1.sh_ptr[gi + 1] - l1.sh_ptr[gi] <= 4;
    std::vector<int32_t> shf4;
    if (fits4) {
      shf4.assign((size_t)4 * l1.nflat_g, -1);
      for (int f = 0; f < l1.nflat_g; ++f) {
        const int gi = l1.gam_iid[f];
        for (int k = l1.sh_ptr[gi]; k < l1.sh_ptr[gi + 1]; ++k) shf4[(size_t)4 * f + (k - l1.sh_ptr[gi])] = l1.sh_flat[k];
      }
    }
    int32_t* sub_flat_d = nullptr;
    const int nblk_avg = std::max(1, (nif + kNT / 8 - 1) / (kNT / 8));   // eight lanes per interface dof
    auto lay = [&] {
      h->partial = B.take<double>(1024);
      P.phi_ptr = B.take<int32_t>(phi_ptr.size());
      P.phi_ids = B.take<int32_t>(nphi);
      P.phi_w = B.take<double>(nphi);
      sub_flat_d = B.take<int32_t>(sub_of_flat.size());
      if (fits4) P.shf4 = B.take<int4>(l1.nflat_g);
      P.Sp = B.take<double>(std::max<size_t>(1, (size_t)spoff.back()));
      P.spoff = B.take<int64_t>(spoff.size());
      P.tpoff = B.take<int64_t>(tpoff.size());
      if (h->precision == BDDC_FP64) P.Tp = B.take<double>(std::max<size_t>(1, (size_t)tpoff.back()));
      if (h->precision != BDDC_FP64) {
        P.Psi32 = B.take<float>((size_t)l1.psioff.back());
        if (h->precision == BDDC_FP32) {
          P.Tp32 = B.take<float>(std::max<size_t>(1, (size_t)tpoff.back()));
        } else {
          P.W16 = B.take<uint16_t>((size_t)l1.toff.back());
          P.Q32 = B.take<float>(std::max<size_t>(1, (size_t)l1.croff.back()));
          P.Dinv = B.take<float>(l1.nflat_g);
        }
      }
    };
    B.reset_sizing();
    lay();
    B.allocate(h->stream);
    lay();
    P.nblk = nblk_avg;
    P.nif = nif;
    P.nsub1 = l1.nsub;
    P.npq = l1.nsub * std::max(1, P.nrb);
    ensure_columns(h, 1);
    {
      // sum the PCG partials once, in a one-block launch, when the consuming
      // blocks would each re-read more than a thousand of them
      // (BDDC_PCG_FINALIZE=0/1/2 forces a form)
      const char* env = getenv("BDDC_PCG_FINALIZE");
      P.fin = env ? std::atoi(env) : (std::max(nblk_avg, l1.nsub) > 1024 ? 1 : 0);
      if (P.fin < 0 || P.fin > 3) P.fin = 1;
      if (P.nrb) P.fin = 1;   // (the row-block launches read the summed scalars)
      // XCD-aware substructure order of the product and update launches
      // (BDDC_XCD_MAP=0/1)
      const char* xe = getenv("BDDC_XCD_MAP");
      P.xcd = xe ? (std::string(xe) == "1" ? 1 : 0) : 1;
    }
    {
      Staging stg(h->stream, &h->staged);
      stg.add(const_cast<int32_t*>(P.phi_ptr), phi_ptr);
      stg.add(sub_flat_d, sub_of_flat);
      if (fits4) stg.add(reinterpret_cast<int32_t*>(const_cast<int4*>(P.shf4)), shf4);
      stg.add(const_cast<int64_t*>(P.spoff), spoff);
      stg.add(const_cast<int64_t*>(P.tpoff), tpoff);
      stg.flush();
      P.prec = h->precision == BDDC_FP32 ? 1 : (h->precision == BDDC_BF16 ? 2 : 0);
      P.ncr = l1.d.ncr;
      P.croff = l1.d.croff;
      int ncrmax = 0;
      for (int v : l1.ncr) ncrmax = std::max(ncrmax, v);
      launch_pack_pcg(h->stream, l1.dev, P);
      launch_round_factors(h->stream, l1.dev, P, l1.nrmax, ncrmax, l1.d.Cr, h->status);
      launch_build_phi(h->stream, l1.dev, nif, sub_flat_d, P.phi_ptr, const_cast<int32_t*>(P.phi_ids),
                       const_cast<double*>(P.phi_w), P.Psi32);
    }
    P.nsub1 = l1.nsub;
    {
      double nshare = 0;
      for (int gi = 0; gi < nif; ++gi) nshare += l1.sh_ptr[gi + 1] - l1.sh_ptr[gi];
      // per interface dof: sharer indices and delta T g, phi row (id, weight, u_c), z and r
      h->by_average = 12.0 * nshare + 20.0 * (double)nphi + 8.0 * nif * 4;
    }
    {
      // the restriction's operator bytes in the storage of the precision form
      double op64 = 0, opp = 0, s64 = 0, sp = 0;
      for (int s = 0; s < l1.nsub; ++s) {
        const double nr = l1.topo.n_r[s], ng = l1.topo.ngam(s), ncs = l1.coff[s + 1] - l1.coff[s];
        const double ncr = l1.ncr[s];
        op64 += 8 * nr * nr + 8 * ng * ncs;
        if (P.prec == 1) opp += 4 * nr * (nr + 1) / 2 + 4 * ng * ncs;
        else if (P.prec == 2) opp += 2 * nr * (nr + 1) / 2 + 4 * nr * ncr + 4 * nr + 4 * ng * ncs;
        else opp += 8 * nr * (nr + 1) / 2 + 8 * ng * ncs;
        s64 += 8 * ng * ng;
        sp += 8 * ng * (ng + 1) / 2;
      }
      h->by_ur_prec = l1.by_update_restrict - op64 + opp;
      h->by_r_prec = l1.by_restrict_ir - op64 + opp;
      h->by_schur_packed = l1.by_schur - s64 + sp;
    }
    clk.lap("pcg state + phi");
    plan_deep(h);
    clk.lap("plan deep");
    Builder::finish(h);
    clk.lap("finish");
    h->sc_host = static_cast<PcgScalars*>(pinned_acquire(sizeof(PcgScalars) * kMaxRhs));
    // info
    std::memset(&h->info, 0, sizeof(h->info));
    h->info.n_free = h->n_free;
    h->info.levels = h->L;
    double ind = h->constraints == BDDC_ADAPTIVE ? 1.0 : 0.0;
    size_t dev = 0;
    for (size_t i = 0; i < h->levels.size(); ++i) {
      fill_level_info(*h->levels[i], (int)i, &h->info);
      if (h->constraints == BDDC_ADAPTIVE) ind *= h->levels[i]->omega;
      dev += h->levels[i]->arena_a.size() + h->levels[i]->arena_b.size() + h->levels[i]->arena_pcg.size();
    }
    h->info.indicator = ind;
    h->info.device_bytes = (int64_t)(dev + h->top.size() + h->coop_arena.size() + h->wide_arena.size());
    h->info.apply_bytes = model_bytes(h, true);
    h->info.matvec_bytes = model_bytes(h, false);
    // a launch configuration the autotuner chose for this shape before
    h->shape_key = shape_key(h);
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      const auto it = g_tune_cache.find(h->shape_key);
      bool valid = it != g_tune_cache.end();
      if (valid) {
        // (a set-up of the same shape may still plan other launches, e.g.
        // forced row blocks; then the remembered choice is not taken)
        try {
          check_tuning(h, it->second);
        } catch (const Error&) {
          valid = false;
        }
      }
      if (valid) {
        apply_tuning(h, it->second);
        h->tuned_ms = it->second.solve_ms;
      }
    }
    h->counted = true;
    g_live_handles.fetch_add(1);
    *out = h;
  });
  if (st != BDDC_OK && h) {
    release(h);
    if (out) *out = nullptr;
  }
  return st;
}


bddc_status bddc_get_tuning(bddc_handle h, bddc_tuning* t) {
  return guard([&] {
    if (!h || !t) fail(BDDC_EINVAL, "handle or tuning is NULL");
    *t = current_tuning(h);
  });
}

bddc_status bddc_set_tuning(bddc_handle h, const bddc_tuning* t) {
  return guard([&] {
    if (!h || !t) fail(BDDC_EINVAL, "handle or tuning is NULL");
    check_tuning(h, *t);
    apply_tuning(h, *t);
    h->tuned_ms = 0.0;
  });
}

bddc_status bddc_autotune(bddc_handle h, const double* f, double* u, int32_t nrhs, int64_t ld, double rtol,
                          int32_t reps, bddc_tuning* t, void* hip_stream) {
  bool noconv = false;
  bddc_status st = guard([&] {
    if (!h || !f || !u || nrhs < 1 || ld < h->n_free || !(rtol >= 0) || reps < 1)
      fail(BDDC_EINVAL, "bad autotune arguments");
    if (h->run.active) fail(BDDC_EBUSY, "a stepwise solve is in progress on this handle");
    hipStream_t saved = h->stream;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    struct Restore {
      bddc_ctx* h;
      hipStream_t s;
      ~Restore() { h->stream = s; }
    } restore{h, saved};
    const int R = std::min<int>(nrhs, kMaxRhs);
    std::vector<int32_t> its(R);
    std::vector<double> rel(R);
    const int maxit = 1000;
    auto solve_once = [&] {
      if (pcg_block(h, f, u, ld, R, rtol, maxit, its.data(), rel.data()) > 0) noconv = true;
    };
    auto time_solves = [&] {
      solve_once();   // first use of a configuration (graph capture) is not timed
      std::vector<double> ms(reps);
      for (int r = 0; r < reps; ++r) {
        const auto t0 = std::chrono::steady_clock::now();
        solve_once();   // synchronises the stream before it returns
        ms[r] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      }
      std::nth_element(ms.begin(), ms.begin() + reps / 2, ms.end());
      return ms[reps / 2];
    };
    bddc_tuning best = current_tuning(h);
    double best_ms = time_solves();
    // one knob at a time; a candidate must win by 2% (timing noise)
    auto try_knob = [&](int bddc_tuning::*knob, std::initializer_list<int> values) {
      for (int v : values) {
        if (v == best.*knob) continue;
        bddc_tuning c = best;
        c.*knob = v;
        if (knob == &bddc_tuning::deep_path && !(deep_available(h) >> v & 1)) continue;
        apply_tuning(h, c);
        const double ms = time_solves();
        if (ms < 0.98 * best_ms) {
          best = c;
          best_ms = ms;
        }
      }
      apply_tuning(h, best);
    };
    try_knob(&bddc_tuning::deep_path, {BDDC_DEEP_COOP, BDDC_DEEP_WIDE, BDDC_DEEP_FUSED, BDDC_DEEP_LEVELS});
    if (!h->pcg.nrb) try_knob(&bddc_tuning::finalize, {0, 1, 2, 3});
    try_knob(&bddc_tuning::check, {4, 8, 16});
    try_knob(&bddc_tuning::graph, {1, 0});
    h->tuned_ms = best_ms;
    best.solve_ms = best_ms;
    best.available = deep_available(h);
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune_cache[h->shape_key] = best;
    }
    if (t) *t = best;
  });
  if (st == BDDC_OK && noconv) return BDDC_ENOCONV;
  return st;
}

bddc_status bddc_apply(bddc_handle h, const double* r, double* z, int32_t nrhs, int64_t ld, void* hip_stream) {
  return guard([&] {
    if (!h || !r || !z || nrhs < 0 || ld < h->n_free) fail(BDDC_EINVAL, "bad apply arguments");
    if (h->run.active) fail(BDDC_EBUSY, "a stepwise solve is in progress on this handle");
    if (r == z) fail(BDDC_EINVAL, "r and z must not alias");
    hipStream_t saved = h->stream;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    for (int c = 0; c < nrhs; ++c) apply_full(h, r + (size_t)c * ld, z + (size_t)c * ld);
    h->stream = saved;
  });
}

bddc_status bddc_solve(bddc_handle h, const double* f, double* u, int32_t nrhs, int64_t ld, double rtol,
                       int32_t maxit, int32_t* iters, double* relres, void* hip_stream) {
  bool noconv = false;
  bddc_status st = guard([&] {
    if (!h || !f || !u || nrhs < 0 || ld < h->n_free || !(rtol >= 0) || maxit < 0 || !iters || !relres)
      fail(BDDC_EINVAL, "bad solve arguments");
    if (maxit > kMaxHist) fail(BDDC_EINVAL, "maxit too large");
    if (h->run.active) fail(BDDC_EBUSY, "a stepwise solve is in progress on this handle");
    hipStream_t saved = h->stream;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    // blocks of up to kMaxRhs columns (BDDC_SOLVE_BLOCK=1: one column at a time)
    const char* env = getenv("BDDC_SOLVE_BLOCK");
    const int blk = env ? std::max(1, std::min(kMaxRhs, atoi(env))) : kMaxRhs;
    for (int c = 0; c < nrhs; c += blk) {
      const int R = std::min(blk, nrhs - c);
      if (pcg_block(h, f + (size_t)c * ld, u + (size_t)c * ld, ld, R, rtol, maxit, iters + c, relres + c) > 0)
        noconv = true;
    }
    h->stream = saved;
  });
  if (st == BDDC_OK && noconv) return BDDC_ENOCONV;
  return st;
}

bddc_status bddc_solve_begin(bddc_handle h, const double* f, int32_t nrhs, int64_t ld, double rtol, int32_t maxit,
                             void* hip_stream) {
  return guard([&] {
    if (!h || !f || nrhs < 1 || nrhs > kMaxRhs || ld < h->n_free || !(rtol >= 0) || maxit < 0)
      fail(BDDC_EINVAL, "bad solve arguments");
    if (maxit > kMaxHist) fail(BDDC_EINVAL, "maxit too large");
    if (h->run.active) fail(BDDC_EBUSY, "a solve is already in progress on this handle");
    const hipStream_t saved = h->stream;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    try {
      pcg_begin(h, f, ld, nrhs, rtol, maxit);
    } catch (...) {
      for (auto& lvp : h->levels) lvp->dev.stop = nullptr;
      h->run.active = false;
      h->stream = saved;
      throw;
    }
    h->run.stepwise = true;
    h->run.saved_stream = saved;
  });
}

static void end_stepwise(bddc_ctx* h) {
  for (auto& lvp : h->levels) lvp->dev.stop = nullptr;
  h->run.active = false;
  h->run.stepwise = false;
  h->stream = h->run.saved_stream;
}

bddc_status bddc_solve_advance(bddc_handle h, int32_t iterations) {
  return guard([&] {
    if (!h || iterations < 0) fail(BDDC_EINVAL, "bad advance arguments");
    if (!h->run.active || !h->run.stepwise) fail(BDDC_EINVAL, "no stepwise solve in progress");
    try {
      pcg_advance(h, iterations);
    } catch (...) {
      end_stepwise(h);
      throw;
    }
  });
}

bddc_status bddc_solve_poll(bddc_handle h, int32_t* state) {
  return guard([&] {
    if (!h || !state) fail(BDDC_EINVAL, "bad poll arguments");
    if (!h->run.active || !h->run.stepwise) fail(BDDC_EINVAL, "no stepwise solve in progress");
    if (!h->run_event) {
      *state = 0;   // nothing advanced yet
      return;
    }
    *state = pcg_poll(h, false);
  });
}

bddc_status bddc_solve_end(bddc_handle h, double* u, int64_t ld, int32_t* iters, double* relres) {
  bool noconv = false;
  bddc_status st = guard([&] {
    if (!h || !u || !iters || !relres) fail(BDDC_EINVAL, "bad solve arguments");
    if (!h->run.active || !h->run.stepwise) fail(BDDC_EINVAL, "no stepwise solve in progress");
    if (ld < h->n_free) fail(BDDC_EINVAL, "bad leading dimension");
    struct End {
      bddc_ctx* h;
      ~End() { end_stepwise(h); }
    } end{h};
    if (pcg_finish(h, u, ld, iters, relres) > 0) noconv = true;
  });
  if (st == BDDC_OK && noconv) return BDDC_ENOCONV;
  return st;
}

bddc_status bddc_solve_noalloc(bddc_handle h, const double* f, double* u, int32_t nrhs, int64_t ld, double rtol,
                               int32_t maxit, int32_t* iters, double* relres, void* hip_stream) {
  bool noconv = false;
  bddc_status st = guard([&] {
    if (!h || !f || !u || nrhs < 0 || ld < h->n_free || !(rtol >= 0) || maxit < 0 || !iters || !relres)
      fail(BDDC_EINVAL, "bad solve arguments");
    if (maxit > kMaxHist) fail(BDDC_EINVAL, "maxit too large");
    if (h->run.active) fail(BDDC_EBUSY, "a stepwise solve is in progress on this handle");
    int dev = -1;
    BDDC_HIP(hipGetDevice(&dev));
    if (dev != h->device) fail(BDDC_EINVAL, "the current device is not the handle's device");
    size_t limit = BDDC_NOALLOC_SCRATCH_BYTES;
    if (const char* env = getenv("BDDC_NOALLOC_LIMIT")) {   // a lower limit, for tests of the size check
      const long long v = atoll(env);
      if (v > 0) limit = std::min(limit, (size_t)v);
    }
    // the caller's layout and the captured chunk stay as they are: the state
    // of this call is laid out in the scratch array and put back at the end
    struct Restore {
      bddc_ctx* h;
      PcgDev pcg;
      double *cy, *ct;
      int ld_cy, cols_cap;
      hipStream_t stream;
      ~Restore() {
        h->pcg = pcg;
        h->cy = cy;
        h->ct = ct;
        h->ld_cy = ld_cy;
        h->cols_cap = cols_cap;
        h->stream = stream;
        h->noalloc_now = false;
      }
    } restore{h, h->pcg, h->cy, h->ct, h->ld_cy, h->cols_cap, h->stream};
    // the widest block of columns whose state fits the scratch
    int blk = 0;
    size_t one = 0;
    for (int R = std::min<int>(kMaxRhs, std::max(1, nrhs)); R >= 1 && blk == 0; --R) {
      Arena A;
      A.reset_sizing();
      lay_columns(h, A, R);
      if (R == 1) one = A.used();
      if (A.used() <= limit) blk = R;
    }
    if (blk == 0)
      fail(BDDC_EUNSUPPORTED, "one column of PCG state needs " + std::to_string(one) + " bytes, more than the " +
                                  std::to_string(limit) + " bytes of the no-allocation scratch");
    if (nrhs == 0) return;
    void* base = noalloc_scratch();
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    h->noalloc_now = true;
    Arena A;
    A.reset_sizing();
    lay_columns(h, A, blk);
    const size_t used = A.used();
    A.attach(base);
    lay_columns(h, A, blk);
    A.detach();
    h->cols_cap = blk;
    // earlier calls (any handle) left their state in the array: start from zeros
    launch_zero_bytes(h->stream, base, used);
    for (int c = 0; c < nrhs; c += blk) {
      const int R = std::min(blk, nrhs - c);
      if (pcg_block(h, f + (size_t)c * ld, u + (size_t)c * ld, ld, R, rtol, maxit, iters + c, relres + c) > 0)
        noconv = true;
    }
  });
  if (st == BDDC_OK && noconv) return BDDC_ENOCONV;
  return st;
}

bddc_status bddc_query(bddc_handle h, bddc_info* info) {
  if (!h || !info) return BDDC_EINVAL;
  *info = h->info;
  return BDDC_OK;
}

bddc_status bddc_edge_eigs(bddc_handle h, int32_t level, int32_t edge, double* lam, int32_t cap,
                           int32_t* n_lam, int32_t* n_sel, int32_t* pair, int32_t* n_edge_dofs) {
  if (!h || h->constraints != BDDC_ADAPTIVE || level < 1 || level > (int)h->levels.size()) return BDDC_EINVAL;
  const Level& lv = *h->levels[level - 1];
  if (edge < 0 || edge >= lv.nedge || cap < 0) return BDDC_EINVAL;
  const int ne = lv.edge_ne[edge];
  if (lam)
    for (int i = 0; i < std::min(cap, ne); ++i) lam[i] = lv.lam[lv.lamoff[edge] + i];
  if (n_lam) *n_lam = ne;
  if (n_sel) *n_sel = lv.edge_nsel[edge];
  if (pair) { pair[0] = lv.topo.edge_s[edge]; pair[1] = lv.topo.edge_t[edge]; }
  if (n_edge_dofs) *n_edge_dofs = ne;
  return BDDC_OK;
}

bddc_status bddc_edge_constraints(bddc_handle h, int32_t level, int32_t edge, int32_t* dofs, int32_t cap_dofs,
                                  double* q, int32_t cap_q, int32_t* n_edge_dofs, int32_t* n_cols) {
  if (!h || level < 1 || level > (int)h->levels.size()) return BDDC_EINVAL;
  const Level& lv = *h->levels[level - 1];
  if (edge < 0 || edge >= lv.nedge) return BDDC_EINVAL;
  const int ne = lv.edge_ne[edge];
  const int m = lv.edge_m.empty() ? 0 : lv.edge_m[edge];
  if (n_edge_dofs) *n_edge_dofs = ne;
  if (n_cols) *n_cols = m;
  if (dofs) {
    if (cap_dofs < ne) return BDDC_EINVAL;
    for (int p = 0; p < ne; ++p) dofs[p] = lv.topo.edge_dof[lv.topo.edge_ptr[edge] + p];
  }
  if (q && ne * m > 0) {
    if (cap_q < ne * m) return BDDC_EINVAL;
    // the installed weights stay on the device; read this edge's columns
    return guard([&] {
      BDDC_HIP(hipMemcpyAsync(q, lv.d.Q + lv.qoff[edge], sizeof(double) * ne * m, hipMemcpyDeviceToHost, h->stream));
      BDDC_HIP(hipStreamSynchronize(h->stream));
    });
  }
  return BDDC_OK;
}

bddc_status bddc_corners(bddc_handle h, int32_t level, int32_t* corners, int32_t cap, int32_t* n_corners) {
  if (!h || level < 1 || level > (int)h->levels.size() || cap < 0) return BDDC_EINVAL;
  const std::vector<int32_t>& c = h->levels[level - 1]->topo.corners;
  const int n = (int)c.size();
  if (n_corners) *n_corners = n;
  if (corners) {
    if (cap < n) return BDDC_EINVAL;
    std::copy(c.begin(), c.end(), corners);
  }
  return BDDC_OK;
}

void bddc_destroy(bddc_handle h) { release(h); }

bddc_status bddc_timing_start(const char* kernel, int32_t every) {
  return guard([&] {
    if (every < 1) fail(BDDC_EINVAL, "every must be >= 1");
    std::lock_guard<std::mutex> lk(timing::mu);
    timing::every = every;
    timing::seen = 0;
    for (auto& r : timing::recs) {
      timing::pool.push_back(r.a);
      timing::pool.push_back(r.b);
    }
    timing::recs.clear();
    timing::target = kernel ? kernel : "";
  });
}

bddc_status bddc_timing_stop(double* total_ms, int64_t* launches, double* bytes, double* flops) {
  return guard([&] {
    std::lock_guard<std::mutex> lk(timing::mu);
    double ms = 0, by = 0, fl = 0;
    for (auto& r : timing::recs) {
      BDDC_HIP(hipEventSynchronize(r.b));
      float t = 0;
      BDDC_HIP(hipEventElapsedTime(&t, r.a, r.b));
      ms += t;
      by += r.bytes;
      fl += r.flops;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = (int64_t)timing::recs.size();
    if (bytes) *bytes = by;
    if (flops) *flops = fl;
    for (auto& r : timing::recs) {
      timing::pool.push_back(r.a);
      timing::pool.push_back(r.b);
    }
    timing::recs.clear();
    timing::target.clear();
  });
}

}  // extern "C"
