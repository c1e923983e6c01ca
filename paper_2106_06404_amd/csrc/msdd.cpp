// Host side of the msdd library: input validation, index planning (the
// symbolic part of the setup), the level-by-level setup orchestration, PCG
// and the C ABI declared in include/msdd.h.
//
// Paper sections: 2.1 (additive subspace correction), 2.2 (hierarchical
// decomposition), 2.3 (spectral coarse spaces, partition of unity,
// Dirichlet subspaces), 3.5 (CG bilinear forms and b^1), 4.1 (patch
// matrices), 4.2 (generating systems on coarse levels), 5 (CG stopping rule).
#include "msdd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "host_util.h"
#include "kernels.h"
#include "net.h"

using namespace msdd_host;

namespace {

int host_threads(int work) {
  unsigned hc = std::thread::hardware_concurrency();
  int nt = (int)std::min<unsigned>(hc ? hc : 1, 16);
  return std::max(1, std::min(nt, work));
}

// Worker threads kept for the life of the process (created on first use, never joined),
// shared by the planning loops of every context, so that a setup does not create and join
// its threads loop after loop.  run() executes body(t) on workers t = 1 .. nthr-1 and on
// the caller as t = 0 and returns when all have finished; a caller that finds the workers
// busy (another thread planning at the same time) gets false and runs on threads of its
// own instead.
class HostPool {
 public:
  static HostPool& get() {
    static HostPool* p = new HostPool;  // never destroyed: its threads outlive static exit
    return *p;
  }
  bool run(int nthr, const std::function<void(int)>& body) {
    std::unique_lock<std::mutex> busy(run_mu_, std::try_to_lock);
    if (!busy.owns_lock()) return false;
    while ((int)workers_ < nthr - 1) {
      const int id = ++workers_;
      std::thread([this, id] { loop(id); }).detach();
    }
    {
      std::lock_guard<std::mutex> g(mu_);
      body_ = &body;
      want_ = nthr - 1;
      pending_ = nthr - 1;
      ++gen_;
    }
    cv_.notify_all();
    body(0);
    std::unique_lock<std::mutex> g(mu_);
    done_.wait(g, [&] { return pending_ == 0; });
    body_ = nullptr;
    return true;
  }

 private:
  void loop(int id) {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> g(mu_);
    for (;;) {
      cv_.wait(g, [&] { return gen_ != seen; });
      seen = gen_;
      if (id > want_) continue;  // not needed in this loop
      const std::function<void(int)>* b = body_;
      g.unlock();
      (*b)(id);
      g.lock();
      if (--pending_ == 0) done_.notify_one();
    }
  }
  std::mutex run_mu_, mu_;
  std::condition_variable cv_, done_;
  int workers_ = 0, want_ = 0, pending_ = 0;
  uint64_t gen_ = 0;
  const std::function<void(int)>* body_ = nullptr;
};

// f(i, thread) for i in [0, n) on nthr threads (dynamic schedule); MsddError from a
// worker is rethrown on the caller.
template <class F>
void parallel_for(int n, int nthr, F f) {
  if (nthr <= 1 || n <= 1) {
    for (int i = 0; i < n; ++i) f(i, 0);
    return;
  }
  std::atomic<int> next(0);
  std::vector<MsddError> errs;
  std::mutex mu;
  const std::function<void(int)> body = [&](int t) {
    try {
      int i;
      while ((i = next++) < n) f(i, t);
    } catch (const MsddError& e) {
      std::lock_guard<std::mutex> g(mu);
      errs.push_back(e);
      next = n;
    }
  };
  if (!HostPool::get().run(nthr, body)) {
    std::vector<std::thread> th;
    for (int t = 0; t < nthr; ++t) th.emplace_back(body, t);
    for (auto& x : th) x.join();
  }
  if (!errs.empty()) throw errs.front();
}

// ---------------------------------------------------------------------------
// An element group (a subdomain or a patch): local dofs in ascending global
// order, local indices of every element dof, dof -> (element, slot) incidences.
// ---------------------------------------------------------------------------
struct GroupPlan {
  std::vector<int> dofs;
  std::vector<int32_t> eloc;      // ne*k
  std::vector<int64_t> inc_ptr;   // ndof+1
  std::vector<int32_t> inc_t;     // element position within the group
  std::vector<int32_t> inc_a;     // local node slot
  int bw = 0;
};

GroupPlan plan_group(const int32_t* elems, int64_t ne, const std::vector<int32_t>& ed, int k,
                     std::vector<int>& map) {
  GroupPlan g;
  for (int64_t t = 0; t < ne; ++t) {
    const int32_t* d = &ed[(size_t)elems[t] * k];
    for (int a = 0; a < k; ++a)
      if (d[a] >= 0 && map[d[a]] == -1) {
        map[d[a]] = -2;
        g.dofs.push_back(d[a]);
      }
  }
  std::sort(g.dofs.begin(), g.dofs.end());
  for (size_t r = 0; r < g.dofs.size(); ++r) map[g.dofs[r]] = (int)r;
  g.eloc.resize((size_t)ne * k);
  std::vector<int64_t> cnt(g.dofs.size() + 1, 0);
  for (int64_t t = 0; t < ne; ++t) {
    const int32_t* d = &ed[(size_t)elems[t] * k];
    int lo = 1 << 30, hi = -1;
    for (int a = 0; a < k; ++a) {
      const int l = d[a] >= 0 ? map[d[a]] : -1;
      g.eloc[(size_t)t * k + a] = l;
      if (l >= 0) {
        cnt[l + 1]++;
        lo = std::min(lo, l);
        hi = std::max(hi, l);
      }
    }
    if (hi >= 0) g.bw = std::max(g.bw, hi - lo);
  }
  for (size_t r = 0; r < g.dofs.size(); ++r) cnt[r + 1] += cnt[r];
  g.inc_ptr = cnt;
  g.inc_t.resize(cnt.back());
  g.inc_a.resize(cnt.back());
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t t = 0; t < ne; ++t)
    for (int a = 0; a < k; ++a) {
      const int l = g.eloc[(size_t)t * k + a];
      if (l >= 0) {
        g.inc_t[pos[l]] = (int32_t)t;
        g.inc_a[pos[l]] = a;
        pos[l]++;
      }
    }
  for (int d : g.dofs) map[d] = -1;
  return g;
}

// Concatenated element-group plans uploaded for the gather kernels.
struct GroupSetDev {
  int ngroups = 0;
  int64_t total_rows = 0;
  std::vector<int64_t> h_voff;  // ngroups+1
  std::vector<int32_t> h_n, h_bw;
  DVec<int32_t> row_grp, slot_elem, slot_loc, inc_slot, inc_a, n, bw;
  DVec<int64_t> voff, inc_ptr;
};

void build_groupset(const std::vector<GroupPlan>& G, const std::vector<std::vector<int32_t>>& elems,
                    int k, GroupSetDev& out, hipStream_t s) {
  out.ngroups = (int)G.size();
  out.h_voff.assign(G.size() + 1, 0);
  out.h_n.resize(G.size());
  out.h_bw.resize(G.size());
  std::vector<int64_t> soff(G.size() + 1, 0);
  for (size_t i = 0; i < G.size(); ++i) {
    out.h_voff[i + 1] = out.h_voff[i] + (int64_t)G[i].dofs.size();
    soff[i + 1] = soff[i] + (int64_t)elems[i].size();
    out.h_n[i] = (int32_t)G[i].dofs.size();
    out.h_bw[i] = G[i].bw;
  }
  out.total_rows = out.h_voff.back();
  // every entry of these arrays is written below (they live only until uploaded)
  HostBuf<int32_t> row_grp(out.total_rows), slot_elem(soff.back()), slot_loc(soff.back() * k);
  HostBuf<int64_t> inc_ptr(out.total_rows + 1);
  inc_ptr[0] = 0;
  // incidence offsets per group, then every group fills its own ranges (in parallel)
  std::vector<int64_t> qoff(G.size() + 1, 0);
  for (size_t i = 0; i < G.size(); ++i) qoff[i + 1] = qoff[i] + (int64_t)G[i].inc_t.size();
  HostBuf<int32_t> inc_slot(qoff.back()), inc_a(qoff.back());
  const int ng = (int)G.size();
  parallel_for(ng, host_threads(ng), [&](int i, int) {
    const auto& g = G[i];
    int64_t q = qoff[i];
    for (size_t r = 0; r < g.dofs.size(); ++r) {
      const int64_t gr = out.h_voff[i] + (int64_t)r;
      row_grp[gr] = (int32_t)i;
      for (int64_t e = g.inc_ptr[r]; e < g.inc_ptr[r + 1]; ++e) {
        inc_slot[q] = (int32_t)(soff[i] + g.inc_t[e]);
        inc_a[q] = g.inc_a[e];
        ++q;
      }
      inc_ptr[gr + 1] = q;
    }
    for (size_t t = 0; t < elems[i].size(); ++t) slot_elem[soff[i] + t] = elems[i][t];
    std::copy(g.eloc.begin(), g.eloc.end(), slot_loc.begin() + soff[i] * k);
  });
  out.row_grp.upload_raw(row_grp.p, row_grp.n, s);
  out.slot_elem.upload_raw(slot_elem.p, slot_elem.n, s);
  out.slot_loc.upload_raw(slot_loc.p, slot_loc.n, s);
  out.inc_slot.upload_raw(inc_slot.p, inc_slot.n, s);
  out.inc_a.upload_raw(inc_a.p, inc_a.n, s);
  out.inc_ptr.upload_raw(inc_ptr.p, inc_ptr.n, s);
  out.voff.upload(out.h_voff, s);
  out.n.upload(out.h_n, s);
  out.bw.upload(out.h_bw, s);
  // no wait: the uploads' sources are staged (pinned) or already copied, and the
  // kernels that read them follow on the same stream
}

// ---------------------------------------------------------------------------
// Patch matrices of one level (Sec. 4.1) held on the device.
// ---------------------------------------------------------------------------
struct PatchLevel {
  int np = 0;
  std::vector<std::vector<int32_t>> members;  // sorted subdomain ids of the level
  std::vector<int32_t> M;                     // functions per patch
  std::vector<std::vector<int32_t>> mcol;     // member column offsets
  std::vector<int64_t> pmoff;                 // np+1 offsets into Pm
  DVec<double> Pm;
  DVec<int32_t> dM;
  DVec<int64_t> dpmoff;
  // for coarse projection: children (patches of the finer level)
  std::vector<std::vector<int32_t>> children;
};

struct FineLevel {
  int P = 0;
  GroupSetDev gs;                       // Neumann-space plans
  std::vector<std::vector<int32_t>> elems;
  std::vector<GroupPlan> plans;
  DVec<double> dv;                      // PoU weights (sorted order)
  DVec<double> dw;                      // PoU weight per Dirichlet entry (doff order): the
                                        // restricted additive Schwarz weights
  DVec<double> dg;                      // b^3: weights 1 - dv of the GEVP right-hand side
                                        // (empty for b^1 and b^2, which use dv)
  DVec<int32_t> elem_ov;                // b^2: 1 for overlap elements (else empty)
  DVec<double> band2, ell_val2;         // b^2: the overlap elements' sum, band and ELL
  // weights of the GEVP right-hand side b = D_g M D_g (M = abar, or band2 / ell_val2)
  const double* gw() const { return dg.p ? dg.p : dv.p; }
  // band storage
  std::vector<int64_t> h_boff;
  DVec<int64_t> boff;
  DVec<double> band;                    // Neumann band (FP64)
  int ell_w = 0;
  DVec<int32_t> ell_col;
  DVec<double> ell_val;
  DVec<double> LSc, LSr;                // LDL^T factor of S = abar + sigma*b (column, row layouts)
  // FP32-factor eigensolver (opt-in): sc = diag(S)^{-1/2} per Neumann row, the LDL^T factor
  // of diag(sc) S diag(sc) in single precision, a vector of ones (abar Y through the b
  // product with unit weights)
  bool eig32 = false;
  bool f64_built = false;  // LSc/LSr hold the FP64 factor
  DVec<double> esc, abar_rs;  // abar_rs: compensated row sums of abar (difference form)
  DVec<float> LS32c, LS32r;
  // blocked form of the same factor (per 64-row block: inverse of the diagonal block and
  // the couplings multiplied by it); built when every half-bandwidth is at most 64
  std::vector<int64_t> h_lbo;
  DVec<int64_t> lbo;
  DVec<double> LB;
  bool has_lb = false;
  // Dirichlet
  std::vector<int32_t> h_nd, h_bd, h_rankb;
  std::vector<int64_t> h_doff, h_dboff;
  DVec<int32_t> nd, bd, dpos, dglob, drow_sub, rankb;
  DVec<int> inertia;  // eigenvalues below eta per subdomain (-1: unknown)
  DVec<int64_t> doff, dboff;
  DVec<double> Dband, LDc, LDr;
  DVec<float> LDc32, LDr32;  // single-precision mode: factor of diag(sc) A_i diag(sc)
  DVec<int32_t> seed_id;     // index of the subdomain within its problem (start blocks)
  DVec<int32_t> wpos;  // warm-start frame position per Neumann row (-1 = none)
  DVec<double> dscale;       // sc per Dirichlet dof (single-precision mode)
  // two-sided form of the Dirichlet solves (twist.hip): blocks before the separator of
  // the top and bottom parts, the bottom part's reversed band and LDL^T factor (nB rows
  // per subdomain at toff), and the separator's C^{-1} (b x b at coff)
  bool has_twist = false;    // every subdomain splits (planned at every setup)
  bool twist_built = false;  // factors built (when the tuning asks for the form)
  std::vector<int32_t> h_tnbt, h_tnbb, h_tnB;
  std::vector<int64_t> h_toff, h_coff;
  DVec<int32_t> tnbt, tnbb, tnB;
  DVec<int64_t> toff, coff;
  int tnB_max = 0;
  DVec<double> Tband, TGc, TGr, TCinv;
  DVec<float> TGc32, TGr32, TCinv32;
  int nd_max = 0, bd_max = 0, bw_max = 0, nb_max = 0;
  // sums used for the algorithmic byte / flop counts of the profiler
  double s_nb = 0, s_band = 0, s_nbb = 0, s_nd = 0, s_dband = 0, s_ndbd = 0, s_ndm = 0, s_m = 0;
  // Dirichlet incidence of fine dofs
  DVec<int64_t> dinc_ptr;
  DVec<int32_t> dinc_sub, dinc_q;
  // eigen results
  std::vector<int32_t> m;
  std::vector<std::vector<double>> lam;  // computed lambdas per subdomain (selected + extra)
  std::vector<int64_t> h_phi_off, h_phid_off, h_moff;
  DVec<int64_t> phi_off, phid_off, moff;
  DVec<int32_t> dm;
  DVec<double> Phi, PhiD;
};

struct CoarseLevel {
  int level = 0;  // l
  int P = 0;
  std::vector<int32_t> no, ng, m;
  std::vector<std::vector<int32_t>> children;  // J_{l,i}
  std::vector<int64_t> h_loff, h_yoff, h_moff, h_lamoff, h_own_ptr;
  std::vector<int32_t> h_own_idx;
  DVec<int32_t> dno, dm, own_idx;
  DVec<int64_t> loff, yoff, moff, own_ptr;
  DVec<double> Lo, Inv, Y, lam;
  std::vector<std::vector<double>> h_lam;
  std::vector<int32_t> rank;
  int no_max = 0;
};

struct EigPass {
  int K = 0;
  DVec<double> X, nu, lam, res, res_e;
  DVec<int> mcount;
  std::vector<int> subs;  // subdomains finalised from this pass
};

// Kernel classes timed with HIP events when profiling is on.
enum ProfId {
  PR_NEUMANN = 0,   // Neumann band + ELL assembly
  PR_DIRICHLET,     // Dirichlet extraction from CSR
  PR_CHOL,          // band Cholesky (S and Dirichlet)
  PR_EIG_SOLVE,     // band solves with K right-hand sides (eigensolver)
  PR_EIG_BAPPLY,    // b = D abar D applied to K vectors
  PR_EIG_GRAM,      // Gram matrices
  PR_EIG_RR,        // Rayleigh-Ritz small eigenproblems
  PR_EIG_UPDATE,    // block update + residuals
  PR_PATCH,         // patch matrices and projections
  PR_COARSE,        // coarse assembly, coarse factorisations and inverses, A_0
  PR_SPMV,          // CSR SpMV (+ fused dot)
  PR_VEC,           // PCG vector updates and dot products
  PR_APPLY_FINE,    // finest-level band triangular solves (LDL^T sweeps)
  PR_APPLY_COARSE,  // coarse-level solves, restriction, prolongation
  PR_APPLY_GATHER,  // finest-level prolongation + gather
  PR_APPLY_RESTRICT,  // finest-level gather of r + restriction to level L-1
  PR_COARSE_GEVP,     // coarse-level GEVPs on the generating systems
  PR_WARM,            // warm-start network inference (BF16 matrix cores)
  PR_OTHER,
  PR_COUNT
};
static_assert(PR_COUNT == MSDD_NPROF, "profile classes");
const char* kProfNames[PR_COUNT] = {
    "neumann_assemble", "dirichlet_extract", "band_cholesky", "eig_band_solve",
    "eig_bapply", "eig_gram", "eig_rayleigh_ritz", "eig_update", "patch", "coarse",
    "spmv", "pcg_vector", "apply_fine_solve", "apply_coarse", "apply_fine_gather",
    "apply_fine_restrict", "coarse_gevp", "warm_infer", "other"};

struct Profiler {
  bool on = false;
  struct Rec {
    int id;
    hipEvent_t a, b;
    double bytes, flops;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double ms[PR_COUNT] = {0};
  int64_t cnt[PR_COUNT] = {0};
  double bytes[PR_COUNT] = {0}, flops[PR_COUNT] = {0};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
  }
  void resolve() {
    for (auto& r : recs) {
      HIPCHK(hipEventSynchronize(r.b));
      float t = 0;
      HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
      ms[r.id] += t;
      cnt[r.id] += 1;
      bytes[r.id] += r.bytes;
      flops[r.id] += r.flops;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
  }
  void reset() {
    resolve();
    for (int i = 0; i < PR_COUNT; ++i) ms[i] = 0, cnt[i] = 0, bytes[i] = 0, flops[i] = 0;
  }
  ~Profiler() {
    for (auto& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct msdd_ctx {
  msdd_options opt;
  hipStream_t stream = nullptr;
  std::string err;
  bool ready = false;
  int n_levels = 0;
  int64_t n = 0, nnz = 0;
  int k = 0;
  double eta = 0, sigma = 0;
  DVec<int64_t> rowptr;
  DVec<int32_t> col;
  DVec<double> val;
  int spmv_sg = 8;
  FineLevel F;
  std::vector<CoarseLevel> C;  // C[0] = level L-1, ..., C[L-2] = level 1
  std::vector<int64_t> nlev;   // n_l for l = 0..L
  int n0 = 0;
  DVec<double> A0, A0inv;       // level 0: dense blocks, one per problem
  int n0_blocks = 1, n0_max = 0;
  std::vector<int64_t> h_a0off;
  DVec<int64_t> a0off, z0off;
  DVec<int32_t> n0blk;
  // solve work
  std::vector<DVec<double>> rlev, zlev;  // index l = 0..L-1
  DVec<double> u, r, z, p, q, x, bvec, partial;
  DVec<double> hyb_t, hyb_q;  // hybrid form: residual of the current correction, A z
  // PCG segments (one per problem) and chunks (row ranges inside one segment)
  std::vector<int64_t> h_seg_row;        // nseg+1
  int nseg = 1, nch = 0;
  DVec<int64_t> ch_lo, ch_hi, seg_ch;
  DVec<int32_t> ch_seg;
  DVec<double> segD, hist_d;  // per-segment CG scalars; residual history
  DVec<int> segI;
  size_t hist_cap = 0;        // entries allocated in hist_d
  int* h_segI = nullptr;      // pinned
  std::vector<int> last_iters;
  std::vector<double> last_relres;
  hipStream_t gstream = nullptr;  // capture stream for the iteration graphs
  hipStream_t ustream = nullptr;  // uploads of the patch planning that overlaps the eigensolves
  hipStream_t cstream = nullptr;  // coarse levels of the preconditioner, beside the fine solve
  hipStream_t istream = nullptr;  // inertia counts, beside the setup's factorisations
  hipEvent_t iev = nullptr;
  hipEvent_t cev0 = nullptr, cev1 = nullptr;
  hipEvent_t gev0 = nullptr, gev1 = nullptr;
  hipGraphExec_t gexec = nullptr;
  const double* g_x = nullptr;  // pointers the cached graph was captured with
  const double* g_b = nullptr;
  int g_maxit = -1;
  msdd_stats_t stats;
  std::vector<double> hist;  // ||r_k|| / ||r_0||, k = 0..iters, of the last solve
  Profiler prof;
  int eig_active = 0;  // subdomains running in the eigensolver (last status read)
  // learned warm start (attached with msdd_warm_start for the next setup)
  struct Warm {
    msdd_net* net = nullptr;
    int P = 0;  // 0 = detached
    int n_in = 0, n_pos = 0, m_cap = 0;
    int64_t n_entries = 0;
    DVec<float> x;              // P x n_in features
    std::vector<int32_t> pos;   // frame position per sub_dof entry
    DVec<float> tgt, mask;      // collected training targets of the last setup
    DVec<int> cnt;
    bool have_targets = false;
  } warm;
  std::vector<int32_t> eig_iters;  // per finest-level subdomain, last setup
  // host scratch of the planning, kept between setups (no fresh pages each time)
  std::vector<double> scr_pou;
  std::vector<int32_t> scr_cnt;
  std::vector<int32_t> scr_ecnt;
  // per planning thread: global dof -> local index maps of size n, all -1 between uses
  // (plan_group restores the entries it sets); kept across setups so that the n-sized
  // arrays are not allocated and filled again; marked dirty while a planning pass runs
  std::vector<std::vector<int>> scr_maps;
  bool scr_maps_clean = false;
  std::vector<int64_t> scr_pos;
  // host copies of the setup's index inputs, kept between setups (their storage is reused)
  std::vector<int64_t> in_rowptr, in_sep, in_sdp;
  std::vector<int32_t> in_ed, in_se, in_sd;
  std::vector<double> in_sw;
  msdd_tuning_t tune{};            // launch-shape choices (0 = by shape)
  ~msdd_ctx() {
    if (h_segI) (void)hipHostFree(h_segI);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (gev0) (void)hipEventDestroy(gev0);
    if (gev1) (void)hipEventDestroy(gev1);
    if (gstream) (void)hipStreamDestroy(gstream);
    if (ustream) (void)hipStreamDestroy(ustream);
    if (cev0) (void)hipEventDestroy(cev0);
    if (cev1) (void)hipEventDestroy(cev1);
    if (cstream) (void)hipStreamDestroy(cstream);
    if (istream) (void)hipStreamDestroy(istream);
    if (iev) (void)hipEventDestroy(iev);
  }
};

namespace {

// verbose: print the time since *t0 under a label and restart the clock
void vlog(msdd_ctx* c, const char* what, double* t0);

void set_err(msdd_ctx* c, const std::string& m) {
  if (c) c->err = m;
}

int code_for(msdd_ctx* c, const MsddError& e) {
  set_err(c, e.msg);
  if (c && c->opt.verbose) std::fprintf(stderr, "msdd: %s\n", e.msg.c_str());
  return e.code;
}

void check_status(const std::vector<int>& st, const char* what, const std::vector<int>* ids = nullptr) {
  for (size_t i = 0; i < st.size(); ++i) {
    if (st[i] == ST_NOTSPD)
      throw MsddError{MSDD_ENOTSPD, std::string(what) + ": non-positive pivot in subdomain " +
                                        std::to_string(ids ? (*ids)[i] : (int)i)};
    if (st[i] == ST_BADINPUT)
      throw MsddError{MSDD_EINVAL, std::string(what) + ": entry outside the element structure or NaN in subdomain " +
                                       std::to_string(ids ? (*ids)[i] : (int)i)};
    if (st[i] == ST_NOCONV)
      throw MsddError{MSDD_EEIG, std::string(what) + ": eigensolver did not converge in subdomain " +
                                     std::to_string(ids ? (*ids)[i] : (int)i)};
  }
}

void vlog(msdd_ctx* c, const char* what, double* t0) {
  const double t = now_ms();
  if (c->opt.verbose) std::fprintf(stderr, "msdd:   %-34s %8.2f ms\n", what, t - *t0);
  *t0 = t;
}

// Records HIP events around the launches of one kernel class (when profiling).
struct ProfScope {
  msdd_ctx* c;
  int id;
  double bytes, flops;
  hipStream_t st;  // the stream the scope's kernels are launched on
  hipEvent_t a = nullptr;
  ProfScope(msdd_ctx* c_, int id_, double bytes_ = 0, double flops_ = 0,
            hipStream_t st_ = nullptr)
      : c(c_), id(id_), bytes(bytes_), flops(flops_), st(st_ ? st_ : c_->stream) {
    if (c->prof.on) {
      a = c->prof.get();
      HIPCHK(hipEventRecord(a, st));
    }
  }
  ~ProfScope() {
    if (c->prof.on && a) {
      hipEvent_t b = c->prof.get();
      if (hipEventRecord(b, st) == hipSuccess) c->prof.recs.push_back({id, a, b, bytes, flops});
    }
  }
};

// ---------------------------------------------------------------------------
// Finest level: planning, local matrices, factorizations, eigensolves
// ---------------------------------------------------------------------------
// Per-subdomain planning results (computed in parallel, merged in subdomain order).
struct SubPlan {
  std::vector<double> dv;            // PoU weight per Neumann dof (0 off the Dirichlet set)
  std::vector<double> dg;            // weights of the GEVP right-hand side (b^3: 1 - dv)
  std::vector<int32_t> dpos, dglob;  // Dirichlet dofs: local Neumann index, global dof
  std::vector<int32_t> wpos;         // warm-start frame position per Neumann dof
  std::vector<int32_t> ell_ptr, ell_col;  // local CSR of the Neumann matrix pattern
  int nD = 0, bd = 0, rankb = 0, ell_w = 0;
  std::string err;
};

// largest finest subdomain (Neumann dofs)
constexpr int kMaxLocalDofs = 1 << 24;

// Number of elements containing each dof (deg[d], d < n), with the range check of the
// element dofs (-1 or below n; MsddError otherwise).  Element ranges are counted in parallel,
// each into a private window of the dofs it touches; the windows are then added up per dof
// range.  Elements numbered without locality (windows summing to more than 4 n) are counted
// in one serial pass instead.
std::unique_ptr<int32_t[]> dof_degrees(const std::vector<int32_t>& ed, int64_t n) {
  const int64_t m = (int64_t)ed.size();
  const int T = host_threads((int)std::min<int64_t>(16, (m + 65535) / 65536));
  struct Win {
    int64_t lo = 0, hi = -1, bad = -1;  // dofs lo..hi; first out-of-range entry
    std::vector<int32_t> cnt;
  };
  std::vector<Win> w(T);
  parallel_for(T, T, [&](int t, int) {
    Win& W = w[t];
    int64_t lo = n, hi = -1;
    for (int64_t q = m * t / T; q < m * (t + 1) / T; ++q) {
      const int64_t d = ed[q];
      if (d < -1 || d >= n) {
        W.bad = q;
        return;
      }
      if (d >= 0) {
        lo = std::min(lo, d);
        hi = std::max(hi, d);
      }
    }
    W.lo = lo;
    W.hi = hi;
  });
  int64_t span = 0;
  for (const Win& W : w) {
    REQUIRE(W.bad < 0, "elem_dofs entry out of range");
    span += std::max<int64_t>(0, W.hi - W.lo + 1);
  }
  std::unique_ptr<int32_t[]> deg(new int32_t[std::max<int64_t>(n, 1)]);  // every entry set below
  if (T == 1 || span > 4 * n) {
    std::fill(deg.get(), deg.get() + n, 0);
    for (int64_t q = 0; q < m; ++q)
      if (ed[q] >= 0) deg[ed[q]]++;
    return deg;
  }
  parallel_for(T, T, [&](int t, int) {
    Win& W = w[t];
    if (W.hi < W.lo) return;
    W.cnt.assign(W.hi - W.lo + 1, 0);
    for (int64_t q = m * t / T; q < m * (t + 1) / T; ++q)
      if (ed[q] >= 0) W.cnt[ed[q] - W.lo]++;
  });
  parallel_for(T, T, [&](int r, int) {
    const int64_t a = n * r / T, b = n * (r + 1) / T;
    std::fill(deg.get() + a, deg.get() + b, 0);
    for (const Win& W : w) {
      const int64_t lo = std::max(a, W.lo), hi = std::min(b, W.hi + 1);
      for (int64_t d = lo; d < hi; ++d) deg[d] += W.cnt[d - W.lo];
    }
  });
  return deg;
}

void plan_fine(msdd_ctx* c, int32_t n_elem, const std::vector<int32_t>& ed,
               const std::vector<int64_t>& sep, const std::vector<int32_t>& se,
               const std::vector<int64_t>& sdp, const std::vector<int32_t>& sd,
               const std::vector<double>& sw, const std::vector<int32_t>* wp) {
  FineLevel& F = c->F;
  const int k = c->k;
  const int64_t n = c->n;
  const int P = F.P;
  double tv = now_ms();
  const std::unique_ptr<int32_t[]> deg = dof_degrees(ed, n);
  for (int i = 0; i < P; ++i)
    REQUIRE(sep[i + 1] >= sep[i] && sdp[i + 1] >= sdp[i], "subdomain pointers not monotone");
  {
    const int64_t m = (int64_t)se.size();
    const int nr = host_threads((int)std::min<int64_t>(16, (m + 65535) / 65536));
    std::vector<int64_t> first(nr, -1);
    parallel_for(nr, nr, [&](int t, int) {
      for (int64_t q = m * t / nr; q < m * (t + 1) / nr; ++q)
        if (se[q] < 0 || se[q] >= n_elem) {
          first[t] = q;
          break;
        }
    });
    for (int t = 0; t < nr; ++t) REQUIRE(first[t] < 0, "sub_elem entry out of range");
  }
  F.elems.assign(P, {});
  F.plans.assign(P, {});
  // b^2: elements that belong to more than one subdomain (the overlap elements)
  const int rhs = c->opt.geneo_rhs;
  std::vector<int32_t>& ecount = c->scr_ecnt;
  if (rhs == 2) {
    ecount.assign(n_elem, 0);
    for (int32_t e : se) ecount[e]++;
  }
  std::vector<SubPlan> sp(P);
  const int nthr = host_threads(P);
  std::vector<std::vector<int>>& maps = c->scr_maps;
  if (!c->scr_maps_clean) maps.clear();  // a pass that did not finish may have left entries
  if ((int)maps.size() < nthr) maps.resize(nthr);
  for (auto& mp : maps)
    if (!mp.empty() && (int64_t)mp.size() != n) mp.clear();
  c->scr_maps_clean = false;
  parallel_for(P, nthr, [&](int i, int t) {
    if (maps[t].empty()) maps[t].assign(n, -1);
    SubPlan& S = sp[i];
    std::vector<int32_t> el(se.begin() + sep[i], se.begin() + sep[i + 1]);
    F.plans[i] = plan_group(el.data(), (int64_t)el.size(), ed, k, maps[t]);
    F.elems[i] = std::move(el);
    const GroupPlan& g = F.plans[i];
    const auto& els = F.elems[i];
    // the caller's Neumann dofs must be the free dofs of the subdomain's elements
    const int64_t nd_in = sdp[i + 1] - sdp[i];
    if (nd_in != (int64_t)g.dofs.size()) {
      S.err = "sub_dof of subdomain " + std::to_string(i) + " is not the set of free dofs of its elements";
      return;
    }
    struct DofW {
      int32_t d;
      double w;
      int32_t p;
    };
    std::vector<DofW> dw((size_t)nd_in);
    for (int64_t q = 0; q < nd_in; ++q)
      dw[q] = {sd[sdp[i] + q], sw[sdp[i] + q], wp ? (*wp)[sdp[i] + q] : -1};
    const auto dw_less = [](const DofW& a, const DofW& b) {
      return a.d < b.d || (a.d == b.d && a.w < b.w);
    };
    if (!std::is_sorted(dw.begin(), dw.end(), dw_less)) std::sort(dw.begin(), dw.end(), dw_less);
    const int nb = (int)g.dofs.size();
    std::vector<int32_t> dloc(nb, -1);
    S.dv.resize(nb);
    S.wpos.resize(nb);
    for (int r = 0; r < nb; ++r) {
      S.wpos[r] = dw[r].p;
      if (dw[r].d != g.dofs[r]) {
        S.err = "sub_dof of subdomain " + std::to_string(i) + " is not the set of free dofs of its elements";
        return;
      }
      const double w = dw[r].w;
      if (!std::isfinite(w)) {
        S.err = "non-finite partition-of-unity weight";
        return;
      }
      const int64_t ninc = g.inc_ptr[r + 1] - g.inc_ptr[r];
      // every adjacent element lies in the subdomain, or (cells and faces) every dof
      const bool dir = c->opt.dirichlet_rule == 1 || ninc == deg[g.dofs[r]];
      if (!dir && std::fabs(w) > 1e-14) {
        S.err = "partition of unity does not vanish on the boundary of subdomain " + std::to_string(i);
        return;
      }
      S.dv[r] = dir ? w : 0.0;
      if (dir) {
        dloc[r] = S.nD++;
        S.dpos.push_back(r);
        S.dglob.push_back(g.dofs[r]);
        if (w != 0.0 && rhs == 1) S.rankb++;
      }
    }
    // weights of the GEVP right-hand side and the rank of b (an upper bound for b^2)
    if (rhs == 3) {
      S.dg.resize(nb);
      for (int r = 0; r < nb; ++r) {
        S.dg[r] = 1.0 - S.dv[r];
        if (S.dg[r] != 0.0) S.rankb++;
      }
    } else if (rhs == 2) {
      std::vector<char> touch(nb, 0);  // the dof lies on an overlap element
      for (size_t q = 0; q < els.size(); ++q)
        if (ecount[els[q]] >= 2)
          for (int a = 0; a < k; ++a) {
            const int l = g.eloc[q * k + a];
            if (l >= 0) touch[l] = 1;
          }
      for (int r = 0; r < nb; ++r)
        if (touch[r] && S.dv[r] != 0.0) S.rankb++;
    }
    for (size_t q = 0; q < els.size(); ++q) {
      int lo = 1 << 30, hi = -1;
      for (int a = 0; a < k; ++a) {
        const int l = g.eloc[q * k + a];
        if (l >= 0 && dloc[l] >= 0) {
          lo = std::min(lo, dloc[l]);
          hi = std::max(hi, dloc[l]);
        }
      }
      if (hi >= 0) S.bd = std::max(S.bd, hi - lo);
    }
    // pattern of the Neumann matrix (ELL rows): distinct neighbours via a marker
    std::vector<int32_t> mark(nb, -1);
    S.ell_ptr.assign(nb + 1, 0);
    for (int r = 0; r < nb; ++r) {
      for (int64_t e = g.inc_ptr[r]; e < g.inc_ptr[r + 1]; ++e) {
        const int q = g.inc_t[e];
        for (int a = 0; a < k; ++a) {
          const int l = g.eloc[(size_t)q * k + a];
          if (l >= 0 && mark[l] != r) {
            mark[l] = r;
            S.ell_col.push_back(l);
          }
        }
      }
      S.ell_ptr[r + 1] = (int32_t)S.ell_col.size();
      // a row holds a few distinct neighbours: insertion sort
      int32_t* rc = S.ell_col.data() + S.ell_ptr[r];
      const int len = S.ell_ptr[r + 1] - S.ell_ptr[r];
      for (int a = 1; a < len; ++a) {
        const int32_t v = rc[a];
        int b = a - 1;
        while (b >= 0 && rc[b] > v) {
          rc[b + 1] = rc[b];
          --b;
        }
        rc[b + 1] = v;
      }
      S.ell_w = std::max(S.ell_w, S.ell_ptr[r + 1] - S.ell_ptr[r]);
    }
  });
  c->scr_maps_clean = true;  // every plan_group call restored its entries
  for (int i = 0; i < P; ++i)
    if (!sp[i].err.empty()) throw MsddError{MSDD_EINVAL, sp[i].err};
  vlog(c, "plan: subdomain groups (parallel)", &tv);
  // merge in subdomain order
  F.h_nd.assign(P, 0);
  F.h_bd.assign(P, 0);
  F.h_rankb.assign(P, 0);
  F.h_doff.assign(P + 1, 0);
  F.h_dboff.assign(P + 1, 0);
  F.ell_w = 0;
  std::vector<double>& pou_sum = c->scr_pou;
  std::vector<int32_t>& dcount = c->scr_cnt;
  pou_sum.resize(n);  // zeroed range by range below
  dcount.resize(n);
  // offsets of each subdomain's entries, sizes and maxima (serial, per subdomain)
  std::vector<int64_t> nbo(P + 1, 0), ndo(P + 1, 0);
  for (int i = 0; i < P; ++i) {
    const GroupPlan& g = F.plans[i];
    const SubPlan& S = sp[i];
    nbo[i + 1] = nbo[i] + (int64_t)g.dofs.size();
    ndo[i + 1] = ndo[i] + S.nD;
    F.h_nd[i] = S.nD;
    F.h_bd[i] = S.bd;
    F.h_rankb[i] = S.rankb;
    F.h_doff[i + 1] = F.h_doff[i] + S.nD;
    F.h_dboff[i + 1] = F.h_dboff[i] + (int64_t)S.nD * (S.bd + 1);
    F.nd_max = std::max(F.nd_max, S.nD);
    F.bd_max = std::max(F.bd_max, S.bd);
    F.bw_max = std::max(F.bw_max, g.bw);
    F.nb_max = std::max(F.nb_max, (int)g.dofs.size());
    F.ell_w = std::max(F.ell_w, S.ell_w);
    F.s_nb += (double)g.dofs.size();
    F.s_band += (double)g.dofs.size() * (g.bw + 1);
    F.s_nbb += (double)g.dofs.size() * g.bw;
    F.s_nd += S.nD;
    F.s_dband += (double)S.nD * (S.bd + 1);
    F.s_ndbd += (double)S.nD * S.bd;
  }
  // two-sided Dirichlet solves when every subdomain splits (half-bandwidth below 64 and
  // at least 65 rows past it) and the workgroup's vector and tables fit in LDS
  {
    F.h_tnbt.assign(P, 0);
    F.h_tnbb.assign(P, 0);
    F.h_tnB.assign(P, 0);
    F.h_toff.assign(P + 1, 0);
    F.h_coff.assign(P + 1, 0);
    F.tnB_max = 0;
    bool ok = P > 0 && F.bd_max < 64;
    for (int i = 0; i < P && ok; ++i) {
      int nbt = 0, nbb = 0;
      twist_split(F.h_nd[i], F.h_bd[i], &nbt, &nbb);
      if (nbt <= 0) {
        ok = false;
        break;
      }
      F.h_tnbt[i] = nbt;
      F.h_tnbb[i] = nbb;
      F.h_tnB[i] = 64 * nbb + F.h_bd[i];
      F.tnB_max = std::max(F.tnB_max, F.h_tnB[i]);
      F.h_toff[i + 1] = F.h_toff[i] + (int64_t)F.h_tnB[i] * (F.h_bd[i] + 1);
      F.h_coff[i + 1] = F.h_coff[i] + (int64_t)F.h_bd[i] * F.h_bd[i];
    }
    const size_t elem = c->opt.precision == MSDD_MIXED ? sizeof(float) : sizeof(double);
    F.has_twist = ok && apply_fine_twist_lds(F.nd_max, F.bd_max, elem, false) <= 160 * 1024;
  }
  // local index arithmetic of the eigensolver blocks (n_i x K, K <= 64) stays in 32 bits
  REQUIRE(F.nb_max <= kMaxLocalDofs,
          "a finest subdomain has " + std::to_string(F.nb_max) + " dofs; at most " +
          std::to_string(kMaxLocalDofs) + " are supported (use more subdomains)");
  // the subdomains' weights and Dirichlet index lists, concatenated (upload-only arrays
  // in the pinned staging arena; every entry is written)
  HostBuf<double> h_dv(nbo[P]), h_dw(ndo[P]), h_dg(rhs == 3 ? nbo[P] : 0);
  HostBuf<int32_t> h_wpos(nbo[P]), h_dpos(ndo[P]), h_dglob(ndo[P]);
  parallel_for(P, nthr, [&](int i, int) {
    const SubPlan& S = sp[i];
    std::copy(S.dv.begin(), S.dv.end(), h_dv.begin() + nbo[i]);
    std::copy(S.wpos.begin(), S.wpos.end(), h_wpos.begin() + nbo[i]);
    if (rhs == 3) std::copy(S.dg.begin(), S.dg.end(), h_dg.begin() + nbo[i]);
    std::copy(S.dpos.begin(), S.dpos.end(), h_dpos.begin() + ndo[i]);
    std::copy(S.dglob.begin(), S.dglob.end(), h_dglob.begin() + ndo[i]);
    for (int q = 0; q < S.nD; ++q) h_dw[ndo[i] + q] = S.dv[S.dpos[q]];
  });
  // PoU sums and Dirichlet multiplicities, each thread over a range of dofs and all
  // subdomains in order (each subdomain's dofs are sorted), so every sum runs in subdomain
  // order as a serial loop would
  const int nrange = std::max(1, (int)std::min<int64_t>(nthr, (n + 16383) / 16384));
  auto range_lo = [&](int t) { return (int32_t)((n * (int64_t)t) / nrange); };
  std::vector<int64_t> rtot(nrange + 1, 0);  // Dirichlet memberships per range
  parallel_for(nrange, nrange, [&](int t, int) {
    const int32_t lo = range_lo(t), hi = range_lo(t + 1);
    std::fill(pou_sum.begin() + lo, pou_sum.begin() + hi, 0.0);
    std::fill(dcount.begin() + lo, dcount.begin() + hi, 0);
    for (int i = 0; i < P; ++i) {
      const GroupPlan& g = F.plans[i];
      const SubPlan& S = sp[i];
      auto b0 = std::lower_bound(g.dofs.begin(), g.dofs.end(), lo);
      for (auto it = b0; it != g.dofs.end() && *it < hi; ++it)
        pou_sum[*it] += S.dv[it - g.dofs.begin()];
      auto d0 = std::lower_bound(S.dglob.begin(), S.dglob.end(), lo);
      for (auto it = d0; it != S.dglob.end() && *it < hi; ++it) dcount[*it]++;
    }
    int64_t tot = 0;
    for (int32_t d = lo; d < hi; ++d) {
      REQUIRE(std::fabs(pou_sum[d] - 1.0) <= 1e-12,
              "partition-of-unity weights do not sum to 1 at dof " + std::to_string(d));
      REQUIRE(dcount[d] > 0, "dof " + std::to_string(d) + " lies in no subdomain's Dirichlet space");
      tot += dcount[d];
    }
    rtot[t + 1] = tot;
  });
  // fine dof -> (subdomain, Dirichlet position), in subdomain order
  // (upload-only arrays in the pinned staging arena; every entry is written)
  for (int t = 0; t < nrange; ++t) rtot[t + 1] += rtot[t];
  HostBuf<int64_t> dptr(n + 1);
  dptr[n] = rtot[nrange];
  HostBuf<int32_t> dsub(dptr[n]), dq(dptr[n]);
  {
    std::vector<int64_t>& pos = c->scr_pos;
    pos.resize(n);
    parallel_for(nrange, nrange, [&](int t, int) {  // prefix sums of the memberships
      int64_t run = rtot[t];
      for (int32_t d = range_lo(t); d < range_lo(t + 1); ++d) {
        dptr[d] = run;
        pos[d] = run;
        run += dcount[d];
      }
    });
    parallel_for(nrange, nrange, [&](int t, int) {
      const int32_t lo = range_lo(t), hi = range_lo(t + 1);
      for (int i = 0; i < P; ++i) {
        const SubPlan& S = sp[i];
        auto d0 = std::lower_bound(S.dglob.begin(), S.dglob.end(), lo);
        for (auto it = d0; it != S.dglob.end() && *it < hi; ++it) {
          const int32_t d = *it;
          dsub[pos[d]] = i;
          dq[pos[d]] = (int32_t)(it - S.dglob.begin());
          pos[d]++;
        }
      }
    });
  }
  vlog(c, "plan: merge + PoU check", &tv);
  hipStream_t s = c->stream;
  build_groupset(F.plans, F.elems, k, F.gs, s);
  F.dv.upload_raw(h_dv.p, h_dv.n, s);
  F.dw.upload_raw(h_dw.p, h_dw.n, s);
  if (rhs == 3) F.dg.upload_raw(h_dg.p, h_dg.n, s);
  else F.dg.release();
  if (rhs == 2) {
    std::vector<int32_t> ov(n_elem);
    for (int32_t e = 0; e < n_elem; ++e) ov[e] = ecount[e] >= 2;
    F.elem_ov.upload(ov, s);
  } else {
    F.elem_ov.release();
  }
  F.wpos.upload_raw(h_wpos.p, h_wpos.n, s);
  F.h_boff.assign(P + 1, 0);
  for (int i = 0; i < P; ++i)
    F.h_boff[i + 1] = F.h_boff[i] + (int64_t)F.plans[i].dofs.size() * (F.plans[i].bw + 1);
  // ELL columns, rows padded with -1 (every entry written here; uploaded from the
  // pinned staging space)
  HostBuf<int32_t> ell((size_t)F.gs.total_rows * F.ell_w);
  parallel_for(P, nthr, [&](int i, int) {
    const SubPlan& S = sp[i];
    const int nb = (int)S.ell_ptr.size() - 1;
    for (int r = 0; r < nb; ++r) {
      const int64_t gr = F.gs.h_voff[i] + r;
      int32_t* row = ell.begin() + gr * F.ell_w;
      const int len = S.ell_ptr[r + 1] - S.ell_ptr[r];
      std::copy(S.ell_col.begin() + S.ell_ptr[r], S.ell_col.begin() + S.ell_ptr[r + 1], row);
      std::fill(row + len, row + F.ell_w, -1);
    }
  });
  F.ell_col.upload_raw(ell.p, ell.n, s);
  F.boff.upload(F.h_boff, s);
  HostBuf<int32_t> drow_sub(F.h_doff.back());
  parallel_for(P, nthr, [&](int i, int) {
    std::fill(drow_sub.begin() + F.h_doff[i], drow_sub.begin() + F.h_doff[i + 1], i);
  });
  F.drow_sub.upload_raw(drow_sub.p, drow_sub.n, s);
  F.nd.upload(F.h_nd, s);
  F.bd.upload(F.h_bd, s);
  F.doff.upload(F.h_doff, s);
  F.dboff.upload(F.h_dboff, s);
  if (F.has_twist) {
    F.tnbt.upload(F.h_tnbt, s);
    F.tnbb.upload(F.h_tnbb, s);
    F.tnB.upload(F.h_tnB, s);
    F.toff.upload(F.h_toff, s);
    F.coff.upload(F.h_coff, s);
  }
  F.dpos.upload_raw(h_dpos.p, h_dpos.n, s);
  F.dglob.upload_raw(h_dglob.p, h_dglob.n, s);
  F.rankb.upload(F.h_rankb, s);
  F.dinc_ptr.upload_raw(dptr.p, dptr.n, s);
  F.dinc_sub.upload_raw(dsub.p, dsub.n, s);
  F.dinc_q.upload_raw(dq.p, dq.n, s);
  vlog(c, "plan: uploads (queued)", &tv);
}

// The side stream (default priority, non-blocking) and the two events that fork work
// onto it and join it back, created on first use.
void ensure_side_stream(msdd_ctx* c) {
  if (c->cstream) return;
  HIPCHK(hipStreamCreateWithFlags(&c->cstream, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&c->cev0, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&c->cev1, hipEventDisableTiming));
  HIPCHK(hipStreamCreateWithFlags(&c->istream, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&c->iev, hipEventDisableTiming));
}

// FP64 LDL^T factor of S = abar + sigma*b for the shift-invert eigensolver, and its
// blocked form where the band allows it.  With the single-precision factor it is built
// only when a subdomain falls back to the FP64 iteration.
void build_eig_factor64(msdd_ctx* c, hipStream_t s, int* status) {
  FineLevel& F = c->F;
  const int P = F.P;
  F.LSc.alloc(F.h_boff.back());
  F.LSr.alloc(F.h_boff.back());
  F.LSc.zero(s);
  F.LSr.zero(s);
  {
    ProfScope ps(c, PR_CHOL, F.s_band * 8.0 * 3.0, F.s_nbb * (F.bw_max + 2.0));
    launch_band_cholesky<double>(s, P, nullptr, F.bw_max, F.gs.n.p, F.gs.bw.p, F.boff.p, F.band.p,
                                 F.gs.voff.p, F.gw(), c->sigma, F.boff.p, F.LSc.p, F.LSr.p,
                                 status, F.band2.p);
  }
  HIPCHK(hipGetLastError());
  // the eigensolver's solves use the LDL^T form: row layout in LSr, column layout in LSc
  launch_band_to_ldl<double>(s, P, F.nb_max, F.bw_max, F.gs.n.p, F.gs.bw.p, F.boff.p, F.LSc.p,
                             F.LSr.p);
  HIPCHK(hipGetLastError());
  // the blocked form (about 3.4 times the band factor for half-bandwidths near 40) is
  // built when the band allows it; if its memory cannot be had, the eigensolver uses
  // the band-factor solves instead
  F.has_lb = F.bw_max <= 64;
  if (F.has_lb) {
    F.h_lbo.assign(P + 1, 0);
    for (int i = 0; i < P; ++i) F.h_lbo[i + 1] = F.h_lbo[i] + band_block_doubles(F.gs.h_n[i]);
    try {
      F.LB.alloc(F.h_lbo.back());
    } catch (const MsddError&) {
      F.has_lb = false;
      F.LB.release();
    }
  }
  if (F.has_lb) {
    F.lbo.upload(F.h_lbo, s);
    ProfScope ps(c, PR_CHOL, F.s_band * 8.0 + (double)F.h_lbo.back() * 8.0,
                 (double)F.h_lbo.back() * 1.25 * F.bw_max);
    launch_band_block_build(s, P, F.nb_max, F.bw_max, F.gs.n.p, F.gs.bw.p, F.boff.p, F.LSr.p,
                            F.lbo.p, F.LB.p);
    HIPCHK(hipGetLastError());
  }
  F.f64_built = true;
}

void fine_local_matrices(msdd_ctx* c, const double* d_elem_mat) {
  FineLevel& F = c->F;
  hipStream_t s = c->stream;
  const int P = F.P;
  DVec<int> status;
  status.alloc(P);
  status.zero(s);
  F.band.alloc(F.h_boff.back());
  F.band.zero(s);
  F.ell_val.alloc((size_t)F.gs.total_rows * F.ell_w);
  F.ell_val.zero(s);
  {
  ProfScope ps(c, PR_NEUMANN, F.s_nb * (8.0 + F.ell_w * 12.0) + F.s_band * 8.0);
  if (F.elem_ov.p) {
    F.band2.alloc(F.h_boff.back());
    F.band2.zero(s);
    F.ell_val2.alloc((size_t)F.gs.total_rows * F.ell_w);
    F.ell_val2.zero(s);
  } else {
    F.band2.release();
    F.ell_val2.release();
  }
  launch_neumann_assemble(s, F.gs.total_rows, F.gs.row_grp.p, F.gs.voff.p, F.gs.bw.p, F.boff.p,
                          F.gs.inc_ptr.p, F.gs.inc_slot.p, F.gs.inc_a.p, F.gs.slot_elem.p,
                          F.gs.slot_loc.p, c->k, d_elem_mat, F.band.p, F.ell_w, F.ell_col.p,
                          F.ell_val.p, status.p, F.elem_ov.p, F.band2.p, F.ell_val2.p);
  }
  F.Dband.alloc(F.h_dboff.back());
  F.Dband.zero(s);
  {
  ProfScope ps(c, PR_DIRICHLET, F.s_nd * 9.0 * 12.0 + F.s_dband * 8.0);
  launch_dirichlet_extract(s, F.h_doff.back(), F.drow_sub.p, F.doff.p, F.nd.p, F.bd.p, F.dboff.p,
                           F.dglob.p, c->rowptr.p, c->col.p, c->val.p, F.Dband.p, status.p);
  }
  HIPCHK(hipGetLastError());
  check_status(status.download(s), "local matrix extraction");
  // factorisations: S = abar + sigma * D abar D (eigensolver) and the Dirichlet matrices
  // (preconditioner) are independent and each is latency bound (one workgroup per
  // subdomain): the Dirichlet one runs on the side stream beside the other, joined
  // before the statuses are read (its profile events are recorded on that stream)
  ensure_side_stream(c);
  const hipStream_t s2 = c->cstream;
  DVec<int> st_scale, st_dchol;  // statuses of the Dirichlet path
  st_scale.alloc(P);
  st_dchol.alloc(P);
  st_scale.zero(s);
  st_dchol.zero(s);
  HIPCHK(hipEventRecord(c->cev0, s));
  HIPCHK(hipStreamWaitEvent(s2, c->cev0, 0));
  // the number of eigenvalues below eta of every pencil (Sylvester inertia of
  // abar - eta b), on a third stream beside both factorisations; the eigensolver stops
  // once its selected pairs converge and their count equals it
  HIPCHK(hipStreamWaitEvent(c->istream, c->cev0, 0));
  F.inertia.alloc(P);
  {
  ProfScope ps(c, PR_CHOL, F.s_band * 8.0, F.s_nbb * (F.bw_max + 2.0), c->istream);
  if (c->opt.nev_fixed > 0) {  // a fixed count has no threshold to certify
    std::vector<int> none(P, -1);
    F.inertia.upload(none, c->istream);
  } else {
    launch_band_inertia(c->istream, P, F.bw_max, F.gs.n.p, F.gs.bw.p, F.boff.p, F.band.p,
                        F.gs.voff.p, F.gw(), -c->eta, F.inertia.p, F.band2.p);
  }
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(c->iev, c->istream));
  const bool mixed = c->opt.precision == MSDD_MIXED;
  if (mixed) {
    // single precision: factor diag(sc) A_i diag(sc), sc = diag(A_i)^{-1/2}
    F.dscale.alloc(std::max<int64_t>(F.h_doff.back(), 1));
    launch_band_scale(s2, P, F.nd_max, F.bd_max, F.nd.p, F.bd.p, F.dboff.p, F.doff.p, F.Dband.p,
                      F.dscale.p, st_scale.p);
    HIPCHK(hipGetLastError());
    F.LDc32.alloc(F.h_dboff.back());
    F.LDr32.alloc(F.h_dboff.back());
    F.LDc32.zero(s2);
    F.LDr32.zero(s2);
    {
    ProfScope ps(c, PR_CHOL, F.s_dband * (8.0 + 2.0 * 4.0), F.s_ndbd * (F.bd_max + 2.0), s2);
    launch_band_cholesky<float>(s2, P, nullptr, F.bd_max, F.nd.p, F.bd.p, F.dboff.p, F.Dband.p,
                                nullptr, nullptr, 0.0, F.dboff.p, F.LDc32.p, F.LDr32.p,
                                st_dchol.p);
    }
    HIPCHK(hipGetLastError());
    launch_band_to_ldl<float>(s2, P, F.nd_max, F.bd_max, F.nd.p, F.bd.p, F.dboff.p, F.LDc32.p,
                              F.LDr32.p);
    HIPCHK(hipGetLastError());
  } else {
    F.LDc.alloc(F.h_dboff.back());
    F.LDr.alloc(F.h_dboff.back());
    F.LDc.zero(s2);
    F.LDr.zero(s2);
    {
    ProfScope ps(c, PR_CHOL, F.s_dband * 8.0 * 3.0, F.s_ndbd * (F.bd_max + 2.0), s2);
    launch_band_cholesky<double>(s2, P, nullptr, F.bd_max, F.nd.p, F.bd.p, F.dboff.p, F.Dband.p,
                                 nullptr, nullptr, 0.0, F.dboff.p, F.LDc.p, F.LDr.p, st_dchol.p);
    }
    HIPCHK(hipGetLastError());
    // the apply uses the LDL^T form: row layout in LDr, column layout in place in LDc
    launch_band_to_ldl<double>(s2, P, F.nd_max, F.bd_max, F.nd.p, F.bd.p, F.dboff.p, F.LDc.p,
                               F.LDr.p);
    HIPCHK(hipGetLastError());
  }
  F.twist_built = F.has_twist && c->tune.fine_solve == 3;
  if (F.twist_built) {
    // two-sided solves: the bottom part's reversed band (from the scaled band in single
    // precision), its factor and the separator's C^{-1}
    ProfScope ps(c, PR_CHOL, F.s_dband * (mixed ? 4.0 : 8.0) * 4.0, F.s_ndbd * (F.bd_max + 2.0) * 0.5,
                 s2);
    const int64_t tn = std::max<int64_t>(F.h_toff.back(), 1);
    F.Tband.alloc(tn);
    launch_twist_extract(s2, P, F.tnB_max, F.bd_max, F.nd.p, F.bd.p, F.tnbt.p, F.tnbb.p, F.dboff.p,
                         F.Dband.p, F.toff.p, F.Tband.p);
    const int64_t cn = std::max<int64_t>(F.h_coff.back(), 1);
    if (mixed) {
      F.TGc32.alloc(tn);
      F.TGr32.alloc(tn);
      F.TGc32.zero(s2);
      F.TGr32.zero(s2);
      F.TCinv32.alloc(cn);
      launch_band_cholesky<float>(s2, P, nullptr, F.bd_max, F.tnB.p, F.bd.p, F.toff.p, F.Tband.p,
                                  nullptr, nullptr, 0.0, F.toff.p, F.TGc32.p, F.TGr32.p, st_dchol.p);
      launch_band_to_ldl<float>(s2, P, F.tnB_max, F.bd_max, F.tnB.p, F.bd.p, F.toff.p, F.TGc32.p,
                                F.TGr32.p);
      launch_twist_schur<float>(s2, P, F.nd.p, F.bd.p, F.tnbt.p, F.tnbb.p, F.dboff.p, F.Dband.p,
                                F.LDr32.p, F.toff.p, F.TGr32.p, F.coff.p, F.TCinv32.p, st_dchol.p);
    } else {
      F.TGc.alloc(tn);
      F.TGr.alloc(tn);
      F.TGc.zero(s2);
      F.TGr.zero(s2);
      F.TCinv.alloc(cn);
      launch_band_cholesky<double>(s2, P, nullptr, F.bd_max, F.tnB.p, F.bd.p, F.toff.p, F.Tband.p,
                                   nullptr, nullptr, 0.0, F.toff.p, F.TGc.p, F.TGr.p, st_dchol.p);
      launch_band_to_ldl<double>(s2, P, F.tnB_max, F.bd_max, F.tnB.p, F.bd.p, F.toff.p, F.TGc.p,
                                 F.TGr.p);
      launch_twist_schur<double>(s2, P, F.nd.p, F.bd.p, F.tnbt.p, F.tnbb.p, F.dboff.p, F.Dband.p,
                                 F.LDr.p, F.toff.p, F.TGr.p, F.coff.p, F.TCinv.p, st_dchol.p);
    }
    HIPCHK(hipGetLastError());
  }
  F.eig32 = c->opt.eig_fp32 == 1;
  if (F.eig32) {
    // single-precision factor of diag(sc) S diag(sc): the scaled Neumann band, then the
    // shifted factorisation with the same weights (b = D abar D commutes with the scaling)
    ProfScope ps(c, PR_CHOL, F.s_band * (8.0 * 3.0 + 4.0 * 2.0), F.s_nbb * (F.bw_max + 2.0));
    F.esc.alloc(std::max<int64_t>(F.gs.total_rows, 1));
    DVec<double> sband;
    sband.alloc(std::max<int64_t>(F.h_boff.back(), 1));
    launch_s_diag_scale(s, F.gs.total_rows, F.gs.row_grp.p, F.gs.voff.p, F.boff.p, F.gs.bw.p,
                        F.band.p, F.gw(), c->sigma, F.esc.p, status.p);
    launch_band_scale_sym(s, F.gs.total_rows, F.gs.row_grp.p, F.gs.voff.p, F.boff.p, F.gs.bw.p,
                          F.gs.n.p, F.band.p, F.esc.p, sband.p);
    F.LS32c.alloc(F.h_boff.back());
    F.LS32r.alloc(F.h_boff.back());
    F.LS32c.zero(s);
    F.LS32r.zero(s);
    launch_band_cholesky<float>(s, P, nullptr, F.bw_max, F.gs.n.p, F.gs.bw.p, F.boff.p, sband.p,
                                F.gs.voff.p, F.gw(), c->sigma, F.boff.p, F.LS32c.p, F.LS32r.p,
                                status.p);
    launch_band_to_ldl<float>(s, P, F.nb_max, F.bw_max, F.gs.n.p, F.gs.bw.p, F.boff.p, F.LS32c.p,
                              F.LS32r.p);
    F.abar_rs.alloc(std::max<int64_t>(F.gs.total_rows, 1));
    launch_abar_rowsum(s, F.gs.total_rows, F.ell_w, F.ell_col.p, F.ell_val.p, F.abar_rs.p);
    HIPCHK(hipGetLastError());
    F.has_lb = false;
  }
  if (!F.eig32) build_eig_factor64(c, s, status.p);
  HIPCHK(hipEventRecord(c->cev1, s2));
  HIPCHK(hipStreamWaitEvent(s, c->cev1, 0));
  HIPCHK(hipStreamWaitEvent(s, c->iev, 0));
  check_status(status.download(s), "Cholesky of abar + sigma*b");
  if (mixed) {
    check_status(st_scale.download(s), "Dirichlet matrix diagonal");
    check_status(st_dchol.download(s), "single-precision Cholesky of the scaled Dirichlet matrices");
  } else {
    check_status(st_dchol.download(s), "Cholesky of the Dirichlet matrices");
  }
  HIPCHK(hipStreamSynchronize(s));
}

// Z = b Y for the eigensolver's K columns per subdomain (skipped where status is not
// running): LDS-tiled when the band allows it, else one thread per row from L2.
void eig_bapply(msdd_ctx* c, hipStream_t s, const int64_t* kvoff, int K, const double* Y,
                double* Z, const int* status) {
  FineLevel& F = c->F;
  const double* ev = F.ell_val2.p ? F.ell_val2.p : F.ell_val.p;  // the matrix inside b
  if (launch_bapply_tile(s, F.P, F.nb_max, F.bw_max, F.gs.voff.p, F.gs.n.p, F.gs.bw.p, kvoff, K,
                         F.gw(), F.ell_w, F.ell_col.p, ev, Y, Z, status))
    return;
  launch_bapply_ell(s, F.gs.total_rows, F.gs.row_grp.p, F.gs.voff.p, F.gs.n.p, kvoff, K, F.gw(),
                    F.ell_w, F.ell_col.p, ev, Y, Z, status);
}

// T = abar Y in difference form (rounding error scaled by the differences y_j - y_r, small
// for vectors near the kernel of abar), for S Y = abar Y + sigma b Y
void eig_abar_apply(msdd_ctx* c, hipStream_t s, const int64_t* kvoff, int K, const double* Y,
                    double* T, const int* status) {
  FineLevel& F = c->F;
  launch_abar_diff(s, F.gs.total_rows, F.gs.row_grp.p, F.gs.voff.p, F.gs.n.p, kvoff, K, F.ell_w,
                   F.ell_col.p, F.ell_val.p, F.abar_rs.p, Y, T, status);
}

// Band solves Y = S^{-1} W of the eigensolver (K columns per subdomain, skipped where
// status is not running).  variant: 0 = by shape (blocked in four launches when the
// blocked factor exists), 1..7 = rolling-window / per-column shapes, 8 = blocked in
// one launch, 9 = blocked in four launches (block-diagonal products apart from the chain).
void eig_band_solve(msdd_ctx* c, hipStream_t s, const int64_t* kvoff, int K, const double* W,
                    double* Y, const int* status, int variant) {
  FineLevel& F = c->F;
  if (variant == 0) variant = F.has_lb ? 9 : 0;
  if ((variant == 8 || variant == 9) && F.has_lb) {
    REQUIRE(W != Y, "blocked band solve: right-hand side and solution must be distinct");
    if (variant == 8)
      launch_band_solve_blk(s, F.P, nullptr, F.gs.n.p, F.gs.bw.p, F.lbo.p, F.LB.p, kvoff, K, W,
                            Y, status);
    else
      launch_band_solve_blk4(s, F.P, nullptr, F.nb_max, F.gs.n.p, F.gs.bw.p, F.lbo.p, F.LB.p,
                             kvoff, K, W, Y, status);
    return;
  }
  launch_band_solve_multi<double, double>(s, F.P, nullptr, F.nb_max, F.gs.n.p, F.gs.bw.p,
                                          F.boff.p, F.LSc.p, F.LSr.p, kvoff, K, W, Y, status,
                                          F.bw_max, variant >= 8 ? 0 : variant);
}

// iteration cap of a pass with the single-precision factor (the FP64 iteration needs
// about 10 to 20 on the inclusion workloads; the preconditioned one converges linearly at
// a rate set by the factor's rounding, so a pass that has not finished by then is stalled)
constexpr int EIG32_MAXIT = 64;

void fine_eigensolve(msdd_ctx* c) {
  FineLevel& F = c->F;
  hipStream_t s = c->stream;
  const int P = F.P;
  const msdd_options& o = c->opt;
  int K = o.block <= 16 ? 16 : (o.block <= 32 ? 32 : 64);
  std::vector<int> want(P, 1);  // subdomains still to solve
  std::vector<int> final_pass(P, -1);
  std::vector<int> final_m(P, 0);
  std::vector<std::unique_ptr<EigPass>> passes;
  int restarts = 0, max_it = 0;
  int unconverged = 0, stagnated = 0, first_unconv = -1;
  double res_max = 0.0, rese_max = 0.0;
  F.lam.assign(P, {});
  // learned warm start: the network's block for every subdomain (BF16 inference)
  msdd_net* net = c->warm.P > 0 ? c->warm.net : nullptr;
  const int n_vec = net ? msdd_net_internal::n_vec(net) : 0;
  const int n_pos = c->warm.P > 0 ? c->warm.n_pos : 0;
  DVec<float> yw;
  std::vector<int> warm_ok(P, net ? 1 : 0);
  if (net) {
    yw.alloc((size_t)P * n_vec * n_pos);
    const double ni = msdd_net_internal::n_in(net), nh = msdd_net_internal::n_hidden(net);
    const double no = (double)n_vec * n_pos;
    // bytes: BF16 weights once + features in + FP32 block out; flops: 2 per multiply-add
    ProfScope ps(c, PR_WARM, 2.0 * (ni * nh + nh * nh + nh * no) + 4.0 * P * (ni + no),
                 2.0 * P * (ni * nh + nh * nh + nh * no));
    msdd_net_internal::infer(net, P, c->warm.x.p, yw.p, s);
  }
  std::vector<int> iters_tot(P, 0);
  int fallbacks = 0;
  // single-precision factor: a subdomain whose iteration stops short of its certificate
  // within EIG32_MAXIT is solved again with the FP64 factor (built on first need)
  std::vector<int> e32_ok(P, F.eig32 ? 1 : 0);
  int fallbacks64 = 0;
  while (true) {
    int nwant = 0;
    bool pass32 = F.eig32;
    for (int i = 0; i < P; ++i) {
      nwant += want[i];
      if (want[i] && !e32_ok[i]) pass32 = false;
    }
    if (!nwant) break;
    if (!pass32 && !F.f64_built) {
      DVec<int> st64;
      st64.alloc(P);
      st64.zero(s);
      build_eig_factor64(c, s, st64.p);
      check_status(st64.download(s), "Cholesky of abar + sigma*b");
    }
    auto ps = std::make_unique<EigPass>();
    EigPass& E = *ps;
    E.K = K;
    std::vector<int64_t> kvoff(P + 1, 0);
    for (int i = 0; i < P; ++i) kvoff[i + 1] = kvoff[i] + (int64_t)F.gs.h_n[i] * K;
    DVec<int64_t> dkvoff;
    dkvoff.upload(kvoff, s);
    const size_t tot = kvoff.back();
    DVec<double> BX, Y, Z, SX, GS, GB, Cm, upart;
    // row splits per subdomain of the Gram and update kernels (about 192 rows each)
    const int nsplit = c->tune.eig_splits > 0 ? c->tune.eig_splits
                                              : std::max(1, std::min(8, (F.nb_max + 191) / 192));
    E.X.alloc(tot);
    BX.alloc(tot);
    Y.alloc(tot);
    Z.alloc(tot);
    SX.alloc(tot);
    GS.alloc((size_t)P * nsplit * K * K);
    GB.alloc((size_t)P * nsplit * K * K);
    upart.alloc((size_t)P * nsplit * UPD_PARTS * K);
    Cm.alloc((size_t)P * K * K);
    E.nu.alloc((size_t)P * K);
    E.lam.alloc((size_t)P * K);
    E.res.alloc((size_t)P * K);
    E.res.zero(s);
    E.res_e.alloc((size_t)P * K);
    E.res_e.zero(s);
    E.mcount.alloc(P);
    E.mcount.zero(s);
    DVec<double> nu_prev, normS, gsd;
    nu_prev.alloc((size_t)P * K);
    nu_prev.zero(s);
    // FP32-factor iteration: residual and correction blocks, S Y; N = 0 and S X = 0 on the
    // first iteration (Y = the scaled solve of B X)
    DVec<double> W32a, W32b, SY;
    if (pass32) {
      W32a.alloc(tot);
      W32b.alloc(tot);
      SY.alloc(tot);
      E.nu.zero(s);
      SX.zero(s);
    }
    gsd.alloc((size_t)P * K);
    gsd.zero(s);
    normS.alloc(P);
    launch_row_norm(s, P, F.gs.voff.p, F.ell_w, F.ell_col.p, F.ell_val.p, F.gw(), c->sigma, normS.p,
                    F.ell_val2.p);
    DVec<int> status, iters;
    std::vector<int> st0(P);
    for (int i = 0; i < P; ++i) st0[i] = want[i] ? ST_RUNNING : ST_DONE;
    status.upload(st0, s);
    iters.alloc(P);
    iters.zero(s);
    DVec<int> dwarm;
    if (net) {
      dwarm.upload(warm_ok, s);
      launch_eig_init_warm(s, F.gs.total_rows, F.gs.row_grp.p, F.gs.voff.p, F.gs.n.p, dkvoff.p, K,
                           F.gw(), E.X.p, 0x5eed5eedull + (unsigned long long)K, F.seed_id.p,
                           dwarm.p, yw.p, n_vec, n_pos, F.wpos.p);
    } else {
      launch_eig_init(s, F.gs.total_rows, F.gs.row_grp.p, F.gs.voff.p, F.gs.n.p, dkvoff.p, K,
                      F.gw(), E.X.p, 0x5eed5eedull + (unsigned long long)K, F.seed_id.p);
    }
    eig_bapply(c, s, dkvoff.p, K, E.X.p, BX.p, status.p);
    const int maxit = pass32 ? std::min(o.eig_maxit, EIG32_MAXIT) : o.eig_maxit;
    std::vector<int> st;
    c->eig_active = nwant;
    for (int it = 0; it < maxit; ++it) {
      const double f = (double)c->eig_active / (double)P;  // share of subdomains still running
      {
        ProfScope ps(c, PR_EIG_SOLVE, f * (2.0 * F.s_band * 8.0 + 4.0 * F.s_nb * K * 8.0),
                     f * 4.0 * F.s_nbb * K);
        if (pass32) {
          // Y = X N + diag(sc) M^{-1} diag(sc) (B X - S X N), M the FP32 factor
          launch_eig32_combine(s, 0, P, F.nb_max, F.gs.n.p, F.gs.voff.p, dkvoff.p, K, BX.p, SX.p,
                               E.nu.p, F.esc.p, 0.0, W32a.p, status.p);
          const int v = c->tune.eig_solve >= 1 && c->tune.eig_solve <= 7 ? c->tune.eig_solve : 0;
          launch_band_solve_multi<float, double>(s, P, nullptr, F.nb_max, F.gs.n.p, F.gs.bw.p,
                                                 F.boff.p, F.LS32c.p, F.LS32r.p, dkvoff.p, K,
                                                 W32a.p, W32b.p, status.p, F.bw_max, v);
          launch_eig32_combine(s, 1, P, F.nb_max, F.gs.n.p, F.gs.voff.p, dkvoff.p, K, E.X.p,
                               W32b.p, E.nu.p, F.esc.p, 0.0, Y.p, status.p);
        } else {
          eig_band_solve(c, s, dkvoff.p, K, BX.p, Y.p, status.p, c->tune.eig_solve);
        }
      }
      {
        ProfScope ps(c, PR_EIG_BAPPLY, f * (F.s_nb * F.ell_w * 12.0 + 2.0 * F.s_nb * K * 8.0),
                     f * 2.0 * F.s_nb * F.ell_w * K);
        eig_bapply(c, s, dkvoff.p, K, Y.p, Z.p, status.p);
        if (pass32) {  // S Y = abar Y + sigma Z
          eig_abar_apply(c, s, dkvoff.p, K, Y.p, W32a.p, status.p);
          launch_eig32_combine(s, 2, P, F.nb_max, F.gs.n.p, F.gs.voff.p, dkvoff.p, K, W32a.p,
                               Z.p, E.nu.p, F.esc.p, c->sigma, SY.p, status.p);
        }
      }
      {
        ProfScope ps(c, PR_EIG_GRAM, f * 3.0 * F.s_nb * K * 8.0, f * 4.0 * F.s_nb * K * K);
        launch_gram(s, P, F.gs.n.p, dkvoff.p, K, Y.p, pass32 ? SY.p : BX.p, Z.p, GS.p, GB.p,
                    status.p, nsplit);
      }
      {
        ProfScope ps(c, PR_EIG_RR, c->eig_active * 3.0 * K * K * 8.0, 0.0);
        launch_rayleigh_ritz(s, P, K, GS.p, GB.p, Cm.p, E.nu.p, status.p, nsplit, gsd.p);
      }
      {
        // reads Y, Z, BX and the previous X, SX; writes X, BX, SX
        ProfScope ps(c, PR_EIG_UPDATE, f * 8.0 * F.s_nb * K * 8.0, f * 6.0 * F.s_nb * K * K);
        launch_eig_update(s, P, F.gs.n.p, dkvoff.p, K, Cm.p, E.nu.p, Y.p, Z.p, E.X.p, BX.p, SX.p,
                          c->sigma, c->eta, o.nev_max, o.eig_tol, maxit, status.p, iters.p,
                          E.mcount.p, E.lam.p, E.res.p, 64, F.rankb.p, normS.p, nu_prev.p,
                          upart.p, nsplit, gsd.p, F.inertia.p, o.nev_fixed, o.eig_tol_energy,
                          E.res_e.p, pass32 ? SY.p : nullptr);
      }
      HIPCHK(hipGetLastError());
      if (it >= 3 && (it % 2 == 1 || it == maxit - 1)) {
        st = status.download(s);
        int act = 0;
        for (int i = 0; i < P; ++i) act += st[i] == ST_RUNNING;
        c->eig_active = act;
        if (!act) break;
      }
    }
    st = status.download(s);
    std::vector<int> mc = E.mcount.download(s);
    std::vector<int> itv = iters.download(s);
    std::vector<double> lamv = E.lam.download(s);
    std::vector<double> resv = E.res.download(s);
    std::vector<double> resev = E.res_e.download(s);
    bool grew = false, fell = false;
    for (int i = 0; i < P; ++i) {
      if (!want[i]) continue;
      max_it = std::max(max_it, itv[i]);
      iters_tot[i] += itv[i];
      if (st[i] == ST_GROW && K < 64) {
        grew = true;
        ++restarts;
        continue;  // stays wanted for the next pass
      }
      if (pass32 && st[i] != ST_DONE) {
        e32_ok[i] = 0;
        fell = true;
        ++fallbacks64;
        if (c->opt.verbose)
          std::fprintf(stderr, "msdd: subdomain %d not converged with the FP32 factor (status %d), "
                       "FP64 pass\n", i, st[i]);
        continue;
      }
      if (warm_ok[i] && st[i] != ST_DONE) {
        // the warm-started iteration did not converge: solve again from the random start
        warm_ok[i] = 0;
        fell = true;
        ++fallbacks;
        if (c->opt.verbose)
          std::fprintf(stderr, "msdd: subdomain %d warm start not converged, cold restart\n", i);
        continue;
      }
      if (st[i] == ST_RUNNING || st[i] == ST_NOCONV || st[i] == ST_GROW) {
        // iteration limit (or a block that cannot grow past 64 columns): the count m is
        // not certified, so the coarse space may miss eigenvectors below eta
        ++unconverged;
        if (first_unconv < 0) first_unconv = i;
        if (c->opt.verbose) {
          std::fprintf(stderr, "msdd: subdomain %d not converged (status %d, %d iterations, K %d, m %d):", i,
                       st[i], itv[i], K, mc[i]);
          for (int a = 0; a < std::min(K, mc[i] + 2); ++a)
            std::fprintf(stderr, " [%.10g %.2e]", lamv[(size_t)i * K + a], resv[(size_t)i * K + a]);
          std::fprintf(stderr, "\n");
        }
      } else {
        // selected pairs accepted at the rounding floor rather than at the tolerance
        for (int a = 0; a < std::min(K, mc[i]); ++a)
          if (resv[(size_t)i * K + a] > o.eig_tol ||
              (o.eig_tol_energy > 0 && resev[(size_t)i * K + a] > o.eig_tol_energy))
            ++stagnated;
      }
      want[i] = 0;
      final_pass[i] = (int)passes.size();
      final_m[i] = mc[i];
      E.subs.push_back(i);
      const int ne = std::min(K, mc[i] + 4);
      F.lam[i].assign(lamv.begin() + (size_t)i * K, lamv.begin() + (size_t)i * K + ne);
      for (int a = 0; a < std::min(K, mc[i]); ++a) {
        res_max = std::max(res_max, resv[(size_t)i * K + a]);
        rese_max = std::max(rese_max, resev[(size_t)i * K + a]);
      }
    }
    passes.push_back(std::move(ps));
    if (!grew && !fell) break;
    if (grew) K *= 2;
  }
  c->eig_iters = iters_tot;
  int64_t isum = 0;
  for (int v : iters_tot) isum += v;
  c->stats.eig_iters_sum = isum;
  c->stats.warm_started = net ? P : 0;
  c->stats.warm_fallbacks = fallbacks;
  c->stats.eig_iters_max = max_it;
  c->stats.eig_restarts = restarts;
  c->stats.eig_resid_max = res_max;
  c->stats.eig_energy_resid_max = rese_max;
  c->stats.eig_unconverged = unconverged;
  c->stats.eig_stagnated = stagnated;
  c->stats.eig_fp64_fallbacks = fallbacks64;
  if (unconverged > 0)
    throw MsddError{MSDD_EEIG, "local eigensolver: " + std::to_string(unconverged) +
                                   " finest-level subdomain(s) not converged within eig_maxit "
                                   "(first: subdomain " + std::to_string(first_unconv) + ")"};
  // pooled basis blocks
  F.m = final_m;
  F.s_ndm = 0;
  F.s_m = 0;
  for (int i = 0; i < P; ++i) {
    F.s_ndm += (double)F.h_nd[i] * F.m[i];
    F.s_m += F.m[i];
  }
  F.h_phi_off.assign(P + 1, 0);
  F.h_phid_off.assign(P + 1, 0);
  F.h_moff.assign(P + 1, 0);
  for (int i = 0; i < P; ++i) {
    F.h_phi_off[i + 1] = F.h_phi_off[i] + (int64_t)F.gs.h_n[i] * F.m[i];
    F.h_phid_off[i + 1] = F.h_phid_off[i] + (int64_t)F.h_nd[i] * F.m[i];
    F.h_moff[i + 1] = F.h_moff[i] + F.m[i];
  }
  F.Phi.alloc(std::max<int64_t>(F.h_phi_off.back(), 1));
  F.PhiD.alloc(std::max<int64_t>(F.h_phid_off.back(), 1));
  F.phi_off.upload(F.h_phi_off, s);
  F.phid_off.upload(F.h_phid_off, s);
  F.moff.upload(F.h_moff, s);
  F.dm.upload(F.m, s);
  const int m_cap = c->warm.P > 0 ? c->warm.m_cap : 0;
  if (m_cap > 0) {
    c->warm.tgt.alloc((size_t)P * m_cap * n_pos);
    c->warm.mask.alloc((size_t)P * n_pos);
    c->warm.cnt.alloc(P);
    c->warm.tgt.zero(s);
    c->warm.mask.zero(s);
    c->warm.cnt.zero(s);
  }
  for (size_t pi = 0; pi < passes.size(); ++pi) {
    EigPass& E = *passes[pi];
    std::vector<int> mm(P, 0);
    for (int i : E.subs) mm[i] = F.m[i];
    E.mcount.upload(mm, s);
    std::vector<int64_t> kvoff(P + 1, 0);
    for (int i = 0; i < P; ++i) kvoff[i + 1] = kvoff[i] + (int64_t)F.gs.h_n[i] * E.K;
    DVec<int64_t> dkvoff;
    dkvoff.upload(kvoff, s);
    launch_eig_finalize(s, P, F.gs.n.p, F.gs.voff.p, dkvoff.p, E.K, F.dv.p, E.X.p, E.nu.p,
                        E.mcount.p, F.phi_off.p, F.Phi.p, F.nd.p, F.doff.p, F.dpos.p,
                        F.phid_off.p, F.PhiD.p);
    HIPCHK(hipGetLastError());
    if (m_cap > 0 && !E.subs.empty()) {
      DVec<int> sel;
      sel.upload(E.subs, s);
      launch_warm_targets(s, (int)E.subs.size(), sel.p, F.gs.n.p, F.gs.voff.p, dkvoff.p, E.K,
                          E.X.p, E.mcount.p, m_cap, n_pos, F.wpos.p, c->warm.tgt.p,
                          c->warm.mask.p, c->warm.cnt.p);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(s));
  }
  c->warm.have_targets = m_cap > 0;
}

// ---------------------------------------------------------------------------
// Patches of the finest level and their projections (Sec. 4.1)
// ---------------------------------------------------------------------------
// Symbolic part of the finest-level patches (depends on the subdomain element sets only),
// run on a host thread while the GPU factorises and solves the local eigenproblems; its
// uploads go to the side stream us.
struct PatchPlan {
  std::vector<std::vector<int32_t>> pel;  // elements per patch
  std::vector<GroupPlan> plans;
  GroupSetDev gs;
  std::vector<int64_t> ploc_off;
  std::vector<int32_t> ploc;              // patch dof -> local index in each member
};

void fine_patches_plan(msdd_ctx* c, const std::vector<int32_t>& ed, int32_t n_elem,
                       PatchLevel& PL, PatchPlan& T, hipStream_t us) {
  FineLevel& F = c->F;
  const int k = c->k;
  double tv = now_ms();
  // element -> containing subdomains (CSR, ascending subdomain order)
  std::vector<int32_t> ecnt(n_elem + 1, 0);
  for (int i = 0; i < F.P; ++i)
    for (int32_t e : F.elems[i]) ecnt[e + 1]++;
  for (int32_t e = 0; e < n_elem; ++e) {
    REQUIRE(ecnt[e + 1] > 0, "element " + std::to_string(e) + " belongs to no subdomain");
    ecnt[e + 1] += ecnt[e];
  }
  std::vector<int32_t> esub(ecnt[n_elem]);
  {
    std::vector<int32_t> pos(ecnt.begin(), ecnt.end() - 1);
    for (int i = 0; i < F.P; ++i)
      for (int32_t e : F.elems[i]) esub[pos[e]++] = i;
  }
  // group elements by their subdomain set; patches are numbered by first element
  std::unordered_map<uint64_t, std::vector<int>> key;
  std::vector<std::vector<int32_t>>& pel = T.pel;
  for (int32_t e = 0; e < n_elem; ++e) {
    const int32_t* m0 = esub.data() + ecnt[e];
    const int cnt = ecnt[e + 1] - ecnt[e];
    uint64_t h = 1469598103934665603ull;
    for (int q = 0; q < cnt; ++q) h = (h ^ (uint64_t)(uint32_t)m0[q]) * 1099511628211ull;
    auto& cand = key[h];
    int id = -1;
    for (int c2 : cand) {
      const auto& mm = PL.members[c2];
      if ((int)mm.size() == cnt && std::equal(mm.begin(), mm.end(), m0)) {
        id = c2;
        break;
      }
    }
    if (id < 0) {
      id = (int)pel.size();
      cand.push_back(id);
      pel.push_back({});
      PL.members.emplace_back(m0, m0 + cnt);
    }
    pel[id].push_back(e);
  }
  PL.np = (int)pel.size();
  vlog(c, "patches: element keys", &tv);
  const int nthr = host_threads(PL.np);
  std::vector<std::vector<int>> maps(nthr);
  std::vector<GroupPlan>& plans = T.plans;
  plans.assign(PL.np, GroupPlan());
  parallel_for(PL.np, nthr, [&](int p, int t) {
    if (maps[t].empty()) maps[t].assign(c->n, -1);
    plans[p] = plan_group(pel[p].data(), (int64_t)pel[p].size(), ed, k, maps[t]);
  });
  vlog(c, "patches: group plans", &tv);
  build_groupset(plans, pel, k, T.gs, us);
  vlog(c, "patches: groupset upload", &tv);
  std::vector<int64_t>& ploc_off = T.ploc_off;
  ploc_off.assign(PL.np + 1, 0);
  for (int p = 0; p < PL.np; ++p)
    ploc_off[p + 1] = ploc_off[p] + (int64_t)plans[p].dofs.size() * (int64_t)PL.members[p].size();
  // patch dof -> local index in each member subdomain (-1 outside it)
  std::vector<int32_t>& ploc = T.ploc;
  ploc.assign(ploc_off.back(), -1);
  parallel_for(PL.np, nthr, [&](int p, int) {
    const int nm = (int)PL.members[p].size();
    const auto& pd = plans[p].dofs;
    int32_t* out = ploc.data() + ploc_off[p];
    for (int sidx = 0; sidx < nm; ++sidx) {
      const auto& sdofs = F.plans[PL.members[p][sidx]].dofs;
      // both lists ascending: merge
      size_t q = 0;
      for (size_t r = 0; r < pd.size(); ++r) {
        while (q < sdofs.size() && sdofs[q] < pd[r]) ++q;
        out[r * nm + sidx] = (q < sdofs.size() && sdofs[q] == pd[r]) ? (int32_t)q : -1;
      }
    }
  });
  vlog(c, "patches: member maps", &tv);
}

// Numeric part: member columns (from the selected counts m_j), uploads and the patch
// projections of the coarse basis (Sec. 4.1)
void fine_patches(msdd_ctx* c, const double* d_elem_mat, PatchLevel& PL, PatchPlan& T) {
  FineLevel& F = c->F;
  hipStream_t s = c->stream;
  const int k = c->k;
  double tv = now_ms();
  const std::vector<GroupPlan>& plans = T.plans;
  const GroupSetDev& gs = T.gs;
  PL.M.assign(PL.np, 0);
  PL.mcol.assign(PL.np, {});
  std::vector<int64_t> mem_ptr(PL.np + 1, 0), vpoff(PL.np + 1, 0);
  std::vector<int32_t> mem_sub, mem_col;
  PL.pmoff.assign(PL.np + 1, 0);
  for (int p = 0; p < PL.np; ++p) {
    int M = 0;
    for (int32_t j : PL.members[p]) {
      PL.mcol[p].push_back(M);
      mem_sub.push_back(j);
      mem_col.push_back(M);
      M += F.m[j];
    }
    PL.M[p] = M;
    mem_ptr[p + 1] = (int64_t)mem_sub.size();
    const int64_t nd = (int64_t)plans[p].dofs.size();
    vpoff[p + 1] = vpoff[p] + nd * M;
    PL.pmoff[p + 1] = PL.pmoff[p] + (int64_t)M * M;
  }
  const std::vector<int64_t>& ploc_off = T.ploc_off;
  const std::vector<int32_t>& ploc = T.ploc;
  DVec<int64_t> dmem_ptr, dploc_off, dvpoff;
  DVec<int32_t> dmem_sub, dmem_col, dploc;
  dmem_ptr.upload(mem_ptr, s);
  dploc_off.upload(ploc_off, s);
  dvpoff.upload(vpoff, s);
  dmem_sub.upload(mem_sub, s);
  dmem_col.upload(mem_col, s);
  dploc.upload(ploc, s);
  PL.dM.upload(PL.M, s);
  PL.dpmoff.upload(PL.pmoff, s);
  DVec<double> V, U;
  V.alloc(std::max<int64_t>(vpoff.back(), 1));
  U.alloc(std::max<int64_t>(vpoff.back(), 1));
  PL.Pm.alloc(std::max<int64_t>(PL.pmoff.back(), 1));
  {
  // algorithmic bytes: the members' basis blocks read, the patch matrices written
  ProfScope pscope(c, PR_PATCH, 8.0 * ((double)F.h_phi_off.back() + (double)PL.pmoff.back()));
  launch_patch_gather(s, PL.np, gs.voff.p, PL.dM.p, dmem_ptr.p, dmem_sub.p, dmem_col.p,
                      dploc_off.p, dploc.p, F.gs.n.p, F.dm.p, F.phi_off.p, F.Phi.p, dvpoff.p, V.p);
  launch_patch_av(s, gs.total_rows, gs.row_grp.p, gs.voff.p, PL.dM.p, gs.inc_ptr.p, gs.inc_slot.p,
                  gs.inc_a.p, gs.slot_elem.p, gs.slot_loc.p, k, d_elem_mat, dvpoff.p, V.p, U.p);
  launch_patch_gram(s, PL.np, gs.voff.p, PL.dM.p, dvpoff.p, V.p, U.p, PL.dpmoff.p, PL.Pm.p);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  vlog(c, "patches: upload + kernels", &tv);
}

// Assemble dense coarse matrices: targets = subdomains of the coarser level (or the
// single level-0 target), each from the patches listed for it.
struct AssembleJob {
  std::vector<int32_t> ng;
  std::vector<int64_t> aoff;
  std::vector<int64_t> tp_ptr, tp_map_off;
  std::vector<int32_t> tp_patch, tp_map;
};

void run_assemble(msdd_ctx* c, const AssembleJob& J, const PatchLevel& PL, DVec<double>& A) {
  hipStream_t s = c->stream;
  DVec<int32_t> ng, tp_patch, tp_map;
  DVec<int64_t> aoff, tp_ptr, tp_map_off;
  ng.upload(J.ng, s);
  aoff.upload(J.aoff, s);
  tp_ptr.upload(J.tp_ptr, s);
  tp_map_off.upload(J.tp_map_off, s);
  tp_patch.upload(J.tp_patch, s);
  tp_map.upload(J.tp_map, s);
  A.alloc(std::max<int64_t>(J.aoff.back(), 1));
  {
  // algorithmic bytes: the patch matrices read, the dense coarse matrices written
  ProfScope ps(c, PR_COARSE, 8.0 * ((double)PL.pmoff.back() + (double)J.aoff.back()));
  launch_coarse_assemble(s, (int)J.ng.size(), tp_ptr.p, tp_patch.p, tp_map_off.p, tp_map.p,
                         PL.dM.p, PL.dpmoff.p, PL.Pm.p, ng.p, aoff.p, A.p);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
}

// m of the subdomains of the level that owns the patches' functions
void coarse_level(msdd_ctx* c, int l, const std::vector<int32_t>& par,
                  const std::vector<int32_t>& m_fine_lvl, const std::vector<int64_t>& moff_fine_lvl,
                  PatchLevel& PL, CoarseLevel& CL, PatchLevel& PLnext) {
  hipStream_t s = c->stream;
  const int Pf = (int)m_fine_lvl.size();
  REQUIRE((int)par.size() == Pf, "parent map size mismatch");
  int Pc = 0;
  for (int32_t v : par) {
    REQUIRE(v >= 0, "negative parent index");
    Pc = std::max(Pc, v + 1);
  }
  double tv = now_ms();
  CL.level = l;
  CL.P = Pc;
  CL.children.assign(Pc, {});
  for (int j = 0; j < Pf; ++j) CL.children[par[j]].push_back(j);
  for (int i = 0; i < Pc; ++i) REQUIRE(!CL.children[i].empty(), "coarse subdomain without children");
  // generating systems
  std::vector<std::vector<int32_t>> contrib(Pc);  // patches meeting subdomain i
  for (int p = 0; p < PL.np; ++p) {
    std::vector<int32_t> ps;
    for (int32_t j : PL.members[p]) ps.push_back(par[j]);
    std::sort(ps.begin(), ps.end());
    ps.erase(std::unique(ps.begin(), ps.end()), ps.end());
    for (int32_t i : ps) contrib[i].push_back(p);
  }
  AssembleJob J;
  J.aoff.assign(Pc + 1, 0);
  J.tp_ptr.assign(Pc + 1, 0);
  CL.no.assign(Pc, 0);
  CL.ng.assign(Pc, 0);
  CL.h_own_ptr.assign(Pc + 1, 0);
  CL.h_own_idx.clear();
  std::vector<int32_t> goff(Pf, -1);
  for (int i = 0; i < Pc; ++i) {
    std::vector<int32_t> ghosts;
    for (int p : contrib[i])
      for (int32_t j : PL.members[p])
        if (par[j] != i) ghosts.push_back(j);
    std::sort(ghosts.begin(), ghosts.end());
    ghosts.erase(std::unique(ghosts.begin(), ghosts.end()), ghosts.end());
    int off = 0;
    for (int32_t j : CL.children[i]) {
      goff[j] = off;
      for (int q = 0; q < m_fine_lvl[j]; ++q) CL.h_own_idx.push_back((int32_t)(moff_fine_lvl[j] + q));
      off += m_fine_lvl[j];
    }
    CL.no[i] = off;
    for (int32_t j : ghosts) {
      goff[j] = off;
      off += m_fine_lvl[j];
    }
    CL.ng[i] = off;
    CL.h_own_ptr[i + 1] = (int64_t)CL.h_own_idx.size();
    for (int p : contrib[i]) {
      J.tp_patch.push_back(p);
      J.tp_map_off.push_back((int64_t)J.tp_map.size());
      for (size_t sidx = 0; sidx < PL.members[p].size(); ++sidx) {
        const int32_t j = PL.members[p][sidx];
        for (int q = 0; q < m_fine_lvl[j]; ++q) J.tp_map.push_back(goff[j] + q);
      }
    }
    J.tp_ptr[i + 1] = (int64_t)J.tp_patch.size();
    J.aoff[i + 1] = J.aoff[i] + (int64_t)off * off;
    for (int32_t j : CL.children[i]) goff[j] = -1;
    for (int32_t j : ghosts) goff[j] = -1;
    CL.no_max = std::max(CL.no_max, CL.no[i]);
  }
  J.ng = CL.ng;
  int ng_max = 0;
  for (int v : CL.ng) ng_max = std::max(ng_max, v);
  REQUIRE(ng_max <= 4096, "coarse generating system with more than 4096 functions");
  vlog(c, "coarse: generating-system plan", &tv);
  DVec<double> Abar;
  run_assemble(c, J, PL, Abar);
  vlog(c, "coarse: assemble (upload + kernel)", &tv);
  // GEVP on the generating systems
  std::vector<int64_t> soff(Pc + 1, 0), lamoff(Pc + 1, 0);
  CL.h_loff.assign(Pc + 1, 0);
  for (int i = 0; i < Pc; ++i) {
    const int64_t ng = CL.ng[i], no = CL.no[i], ngh = ng - no;
    // S, Q, Qk, C, Yc (ng^2 each), ints, then d and the eigensolver workspace for
    // generating systems whose workspace does not fit in LDS
    soff[i + 1] = soff[i] + 5 * ng * ng + ng + 2 + coarse_gevp_vec_doubles((int)ng);
    (void)ngh;
    CL.h_loff[i + 1] = CL.h_loff[i] + no * no;
    lamoff[i + 1] = lamoff[i] + no;
  }
  DVec<int32_t> dng, dno;
  DVec<int64_t> dsoff, dlamoff;
  dng.upload(CL.ng, s);
  dno.upload(CL.no, s);
  dsoff.upload(soff, s);
  dlamoff.upload(lamoff, s);
  CL.loff.upload(CL.h_loff, s);
  CL.dno.upload(CL.no, s);
  DVec<double> scratch;
  scratch.alloc(std::max<int64_t>(soff.back(), 1));
  CL.Lo.alloc(std::max<int64_t>(CL.h_loff.back(), 1));
  CL.lam.alloc(std::max<int64_t>(lamoff.back(), 1));
  DVec<int> mo, st, rk, sweeps;
  mo.alloc(Pc);
  st.alloc(Pc);
  rk.alloc(Pc);
  sweeps.alloc(4 * Pc);
  st.zero(s);
  DVec<int64_t> aoff;
  aoff.upload(J.aoff, s);
  std::vector<int> sw;
  std::vector<int> rkh;
  {
    // flops of the two symmetric eigendecompositions (sizes ng and r): Householder
    // tridiagonalisation and accumulation of Q, 8/3 n^3; the divide-and-conquer merges'
    // eigenvector products, 8/3 n^3 (2 s^2 k per merge of width s with k roots, summed
    // over the levels with k = s); the back-transformation Q W, 2 n^3
    ProfScope pscope(c, PR_COARSE_GEVP);
    launch_coarse_gevp(s, Pc, dng.p, dno.p, aoff.p, Abar.p, CL.loff.p, CL.Lo.p, dsoff.p,
                       scratch.p, c->eta, c->opt.nev_max, c->opt.eps_reg_rel, CL.lam.p, dlamoff.p,
                       mo.p, st.p, rk.p, sweeps.p,
                       Pc ? *std::max_element(CL.ng.begin(), CL.ng.end()) : 0);
    HIPCHK(hipGetLastError());
    sw = sweeps.download(s);
    rkh = rk.download(s);
    double fl = 0.0;
    for (int i = 0; i < Pc; ++i)
      for (int q = 0; q < 2; ++q) {
        const double nn = sw[4 * i + 2 + q];
        fl += 22.0 / 3.0 * nn * nn * nn;
      }
    pscope.flops = fl;
  }
  std::vector<int> stv = st.download(s);
  vlog(c, "coarse: GEVP kernel", &tv);
  if (c->opt.verbose) {
    int ngm = 0, rmax = 0;
    for (int i = 0; i < Pc; ++i) {
      ngm = std::max(ngm, CL.ng[i]);
      rmax = std::max(rmax, rkh[i]);
    }
    fprintf(stderr, "msdd:   coarse level %d: %d subdomains, ng max %d, rank max %d\n", l, Pc,
            ngm, rmax);
  }
  check_status(stv, "coarse GEVP (eigensolver or Cholesky of the owned block)");
  CL.m = mo.download(s);
  CL.rank = rk.download(s);
  std::vector<double> lamh = CL.lam.download(s);
  CL.h_lam.assign(Pc, {});
  for (int i = 0; i < Pc; ++i) CL.h_lam[i].assign(lamh.begin() + lamoff[i], lamh.begin() + lamoff[i + 1]);
  CL.h_yoff.assign(Pc + 1, 0);
  CL.h_moff.assign(Pc + 1, 0);
  for (int i = 0; i < Pc; ++i) {
    CL.h_yoff[i + 1] = CL.h_yoff[i] + (int64_t)CL.no[i] * CL.m[i];
    CL.h_moff[i + 1] = CL.h_moff[i] + CL.m[i];
  }
  CL.yoff.upload(CL.h_yoff, s);
  CL.moff.upload(CL.h_moff, s);
  CL.dm.upload(CL.m, s);
  CL.own_ptr.upload(CL.h_own_ptr, s);
  CL.own_idx.upload(CL.h_own_idx, s);
  CL.Y.alloc(std::max<int64_t>(CL.h_yoff.back(), 1));
  launch_coarse_collect(s, Pc, dng.p, dno.p, dsoff.p, scratch.p, CL.dm.p, CL.yoff.p, CL.Y.p);
  {
    DVec<double> Linv;
    Linv.alloc(std::max<int64_t>(CL.h_loff.back(), 1));
    CL.Inv.alloc(std::max<int64_t>(CL.h_loff.back(), 1));
    launch_spd_inverse(s, Pc, CL.no_max, CL.loff.p, CL.dno.p, CL.Lo.p, Linv.p, CL.Inv.p);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  // patches of level l from those of level l+1, grouped by parent sets
  std::map<std::vector<int32_t>, int> key;
  PLnext.members.clear();
  PLnext.children.clear();
  std::vector<int32_t> cpar(PL.np);
  for (int p = 0; p < PL.np; ++p) {
    std::vector<int32_t> ps;
    for (int32_t j : PL.members[p]) ps.push_back(par[j]);
    std::sort(ps.begin(), ps.end());
    ps.erase(std::unique(ps.begin(), ps.end()), ps.end());
    auto it = key.find(ps);
    int id;
    if (it == key.end()) {
      id = (int)PLnext.members.size();
      key.emplace(ps, id);
      PLnext.members.push_back(ps);
      PLnext.children.push_back({});
    } else {
      id = it->second;
    }
    PLnext.children[id].push_back(p);
    cpar[p] = id;
  }
  PLnext.np = (int)PLnext.members.size();
  PLnext.M.assign(PLnext.np, 0);
  PLnext.mcol.assign(PLnext.np, {});
  PLnext.pmoff.assign(PLnext.np + 1, 0);
  std::vector<int64_t> pmem_ptr(PLnext.np + 1, 0), ch_ptr(PLnext.np + 1, 0), wsoff(PLnext.np + 1, 0);
  std::vector<int32_t> pmem_sub, pmem_col, ch_patch;
  for (int q = 0; q < PLnext.np; ++q) {
    int M = 0;
    for (int32_t i : PLnext.members[q]) {
      PLnext.mcol[q].push_back(M);
      pmem_sub.push_back(i);
      pmem_col.push_back(M);
      M += CL.m[i];
    }
    PLnext.M[q] = M;
    pmem_ptr[q + 1] = (int64_t)pmem_sub.size();
    PLnext.pmoff[q + 1] = PLnext.pmoff[q] + (int64_t)M * M;
    int64_t wmax = 0;
    for (int p : PLnext.children[q]) {
      ch_patch.push_back(p);
      wmax = std::max<int64_t>(wmax, (int64_t)PL.M[p] * M);
    }
    ch_ptr[q + 1] = (int64_t)ch_patch.size();
    wsoff[q + 1] = wsoff[q] + wmax;
  }
  // child patch member info: parent slot, position within the parent's owned list
  std::vector<int32_t> ownbase(Pf, 0);
  for (int i = 0; i < Pc; ++i) {
    int off = 0;
    for (int32_t j : CL.children[i]) {
      ownbase[j] = off;
      off += m_fine_lvl[j];
    }
  }
  std::vector<int64_t> cmem_ptr(PL.np + 1, 0);
  std::vector<int32_t> cmem_pslot, cmem_ownbase, cmem_m, cmem_col;
  for (int p = 0; p < PL.np; ++p) {
    const auto& pm = PLnext.members[cpar[p]];
    for (size_t sidx = 0; sidx < PL.members[p].size(); ++sidx) {
      const int32_t j = PL.members[p][sidx];
      const int ps = (int)(std::lower_bound(pm.begin(), pm.end(), par[j]) - pm.begin());
      cmem_pslot.push_back(ps);
      cmem_ownbase.push_back(ownbase[j]);
      cmem_m.push_back(m_fine_lvl[j]);
      cmem_col.push_back(PL.mcol[p][sidx]);
    }
    cmem_ptr[p + 1] = (int64_t)cmem_pslot.size();
  }
  DVec<int64_t> dch_ptr, dcmem_ptr, dpmem_ptr, dwsoff;
  DVec<int32_t> dch_patch, dcmem_pslot, dcmem_ownbase, dcmem_m, dcmem_col, dpmem_sub, dpmem_col;
  dch_ptr.upload(ch_ptr, s);
  dcmem_ptr.upload(cmem_ptr, s);
  dpmem_ptr.upload(pmem_ptr, s);
  dwsoff.upload(wsoff, s);
  dch_patch.upload(ch_patch, s);
  dcmem_pslot.upload(cmem_pslot, s);
  dcmem_ownbase.upload(cmem_ownbase, s);
  dcmem_m.upload(cmem_m, s);
  dcmem_col.upload(cmem_col, s);
  dpmem_sub.upload(pmem_sub, s);
  dpmem_col.upload(pmem_col, s);
  PLnext.dM.upload(PLnext.M, s);
  PLnext.dpmoff.upload(PLnext.pmoff, s);
  PLnext.Pm.alloc(std::max<int64_t>(PLnext.pmoff.back(), 1));
  DVec<double> Wsc;
  Wsc.alloc(std::max<int64_t>(wsoff.back(), 1));
  {
  // algorithmic bytes: this level's patch matrices and owned bases read, the next level's
  // patch matrices written
  ProfScope pscope2(c, PR_PATCH, 8.0 * ((double)PL.pmoff.back() + (double)CL.h_yoff.back() +
                                        (double)PLnext.pmoff.back()));
  vlog(c, "coarse: next-level patch plan", &tv);
  launch_patch_project(s, PLnext.np, dch_ptr.p, dch_patch.p, PL.dM.p, PL.dpmoff.p, PL.Pm.p,
                       dcmem_ptr.p, dcmem_pslot.p, dcmem_ownbase.p, dcmem_m.p, dcmem_col.p,
                       dpmem_ptr.p, dpmem_sub.p, dpmem_col.p, nullptr, CL.dno.p, CL.yoff.p, CL.Y.p,
                       PLnext.dM.p, PLnext.dpmoff.p, PLnext.Pm.p, dwsoff.p, Wsc.p);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  vlog(c, "coarse: patch projection kernel", &tv);
}

// Level 0: one dense block per problem (a single problem: A_0 itself), assembled from
// the patches of level 1 (Sec. 4.1), factorised and inverted.  prob[i] = problem of
// level-1 subdomain i (nondecreasing).
// above this size the coarsest space of a single problem is factorised by tiles over the
// whole device instead of by one workgroup
constexpr int kBlockedCoarsest = 384;

void coarsest(msdd_ctx* c, const PatchLevel& PL, const std::vector<int32_t>& m_lvl1,
              const std::vector<int32_t>& prob, int nprob) {
  hipStream_t s = c->stream;
  const int P1 = (int)m_lvl1.size();
  std::vector<int64_t> moff(P1 + 1, 0);
  for (int i = 0; i < P1; ++i) moff[i + 1] = moff[i] + m_lvl1[i];
  c->n0 = (int)moff.back();
  // per problem: level-0 range [zoff, zoff + n0_t)
  std::vector<int64_t> zoff(nprob + 1, 0);
  {
    std::vector<int64_t> cnt(nprob, 0);
    for (int i = 0; i < P1; ++i) cnt[prob[i]] += m_lvl1[i];
    for (int t = 0; t < nprob; ++t) zoff[t + 1] = zoff[t] + cnt[t];
  }
  AssembleJob J;
  J.ng.resize(nprob);
  J.aoff.assign(nprob + 1, 0);
  int nmax = 0;
  for (int t = 0; t < nprob; ++t) {
    J.ng[t] = (int32_t)(zoff[t + 1] - zoff[t]);
    // one problem: tiled factorisation over the whole device (three n_0^2 matrices);
    // a batch: one workgroup per problem
    REQUIRE(J.ng[t] <= (nprob == 1 ? 32768 : 8192),
            nprob == 1 ? "coarsest space larger than 32768 (add a level)"
                       : "coarsest space of a batch member larger than 8192 (add a level)");
    J.aoff[t + 1] = J.aoff[t] + (int64_t)J.ng[t] * J.ng[t];
    nmax = std::max(nmax, J.ng[t]);
  }
  std::vector<std::vector<int>> tpatch(nprob);
  for (int p = 0; p < PL.np; ++p) {
    const int t = prob[PL.members[p][0]];
    for (int32_t i : PL.members[p]) REQUIRE(prob[i] == t, "a patch spans two problems");
    tpatch[t].push_back(p);
  }
  J.tp_ptr.assign(nprob + 1, 0);
  for (int t = 0; t < nprob; ++t) {
    for (int p : tpatch[t]) {
      J.tp_patch.push_back(p);
      J.tp_map_off.push_back((int64_t)J.tp_map.size());
      for (int32_t i : PL.members[p])
        for (int q = 0; q < m_lvl1[i]; ++q) J.tp_map.push_back((int32_t)(moff[i] + q - zoff[t]));
    }
    J.tp_ptr[t + 1] = (int64_t)J.tp_patch.size();
  }
  c->n0_blocks = nprob;
  c->n0_max = nmax;
  c->h_a0off = J.aoff;
  c->a0off.upload(J.aoff, s);
  c->z0off.upload(zoff, s);
  c->n0blk.upload(J.ng, s);
  if (c->n0 == 0) {
    c->A0.alloc(1);
    c->A0inv.alloc(1);
    return;
  }
  run_assemble(c, J, PL, c->A0);
  if (nprob == 1 && nmax > kBlockedCoarsest) {
    // factor, L^{-1} and the explicit inverse by 64 x 64 tiles over every compute unit
    std::vector<int> ok(1, ST_DONE);
    DVec<int> st;
    st.upload(ok, s);
    DVec<double> Linv;
    Linv.alloc((size_t)nmax * nmax);
    c->A0inv.alloc((size_t)nmax * nmax);
    const double nn = (double)nmax;
    {
      ProfScope ps(c, PR_COARSE, 6.0 * nn * nn * 8.0, nn * nn * nn);
      launch_blocked_spd_inverse(s, nmax, c->A0.p, Linv.p, c->A0inv.p, st.p);
    }
    HIPCHK(hipGetLastError());
    if (st.download(s)[0] != ST_DONE)
      throw MsddError{MSDD_ENOTSPD, "coarsest matrix A_0 is not positive definite"};
    HIPCHK(hipStreamSynchronize(s));
    return;
  }
  DVec<int> st;
  st.alloc(nprob);
  double fl = 0.0, by = 0.0;
  for (int t = 0; t < nprob; ++t) {
    fl += (double)J.ng[t] * J.ng[t] * J.ng[t] / 3.0;
    by += 2.0 * J.ng[t] * (double)J.ng[t] * 8.0;
  }
  {
    ProfScope ps(c, PR_COARSE, by, fl);
    launch_dense_cholesky(s, nprob, nmax, c->a0off.p, c->n0blk.p, c->A0.p, st.p);
  }
  HIPCHK(hipGetLastError());
  std::vector<int> v = st.download(s);
  for (int t = 0; t < nprob; ++t)
    if (v[t] != ST_DONE)
      throw MsddError{MSDD_ENOTSPD, "coarsest matrix A_0 of problem " + std::to_string(t) +
                                        " is not positive definite"};
  {
    DVec<double> Linv;
    Linv.alloc((size_t)J.aoff.back());
    c->A0inv.alloc((size_t)J.aoff.back());
    ProfScope ps(c, PR_COARSE, 1.5 * by, 2.0 * fl);
    launch_spd_inverse(s, nprob, nmax, c->a0off.p, c->n0blk.p, c->A0.p, Linv.p, c->A0inv.p);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
}

void alloc_solve_work(msdd_ctx* c) {
  const int L = c->n_levels - 1;
  c->rlev.clear();
  c->zlev.clear();
  c->rlev.resize(L);
  c->zlev.resize(L);
  for (int l = 0; l < L; ++l) {
    c->rlev[l].alloc(std::max<int64_t>(c->nlev[l], 1));
    c->zlev[l].alloc(std::max<int64_t>(c->nlev[l], 1));
  }
  c->u.alloc(std::max<int64_t>(c->F.h_doff.back(), 1));
  const int64_t n = c->n;
  c->r.alloc(n);
  c->z.alloc(n);
  c->p.alloc(n);
  c->q.alloc(n);
  c->x.alloc(n);
  c->bvec.alloc(n);
  c->hyb_t.alloc(n);
  c->hyb_q.alloc(n);
  // chunks of at most 256 rows, never crossing a segment boundary
  const int64_t CH = 256;
  std::vector<int64_t> lo, hi, sch(c->nseg + 1, 0);
  std::vector<int32_t> sg;
  for (int q = 0; q < c->nseg; ++q) {
    for (int64_t a = c->h_seg_row[q]; a < c->h_seg_row[q + 1]; a += CH) {
      lo.push_back(a);
      hi.push_back(std::min(a + CH, c->h_seg_row[q + 1]));
      sg.push_back(q);
    }
    sch[q + 1] = (int64_t)lo.size();
  }
  c->nch = (int)lo.size();
  hipStream_t s = c->stream;
  c->ch_lo.upload(lo, s);
  c->ch_hi.upload(hi, s);
  c->ch_seg.upload(sg, s);
  c->seg_ch.upload(sch, s);
  c->partial.alloc(std::max(c->nch, 1));
  c->segD.alloc((size_t)c->nseg * PCG_SD);
  c->segI.alloc((size_t)c->nseg * PCG_SI);
  if (c->h_segI) (void)hipHostFree(c->h_segI);
  c->h_segI = nullptr;
  HIPCHK(hipHostMalloc((void**)&c->h_segI, (size_t)c->nseg * PCG_SI * sizeof(int), hipHostMallocDefault));
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
  c->hist_d.release();
  c->hist_cap = 0;
  HIPCHK(hipStreamSynchronize(s));
}

// z = B r (Sec. 2.1, additive over all levels), launched on stream s.  After the
// restriction the coarse levels (a chain of small launches) and the finest-level solves
// are independent: without profiling the coarse chain runs on a second stream, forked
// and joined with events (inside a captured iteration graph these become graph edges),
// so that it overlaps the solves.
// Algorithmic work of the coarse part of one preconditioner apply: per coarse level the
// owned blocks' inverses (no_i^2) and the basis blocks (no_i m_i, read on the way down and
// up), the vectors they touch, and the coarsest inverse (n_0^2 per problem).
static void apply_coarse_work(const msdd_ctx* c, double* bytes, double* flops) {
  double by = 0, fl = 0;
  for (const CoarseLevel& CL : c->C) {
    const double inv = CL.h_loff.empty() ? 0.0 : (double)CL.h_loff.back();
    const double y = CL.h_yoff.empty() ? 0.0 : (double)CL.h_yoff.back();
    const double no = CL.h_own_ptr.empty() ? 0.0 : (double)CL.h_own_ptr.back();
    const double m = CL.h_moff.empty() ? 0.0 : (double)CL.h_moff.back();
    by += 8.0 * (inv + 2.0 * y + 4.0 * no + 2.0 * m) + 8.0 * no;  // + the owned indices
    fl += 2.0 * inv + 4.0 * y;
  }
  const double a0 = c->h_a0off.empty() ? 0.0 : (double)c->h_a0off.back();
  by += 8.0 * a0;
  fl += 2.0 * a0;
  *bytes = by;
  *flops = fl;
}

// The finest-level local solves u_i = A_i^{-1} u_i.  variant: 0 = by shape (the rolling
// window for half-bandwidths below 64, else one wavefront), 1 = rolling window, 2 = one
// wavefront per subdomain, 3 = two-sided (when its factors were built at the setup, else
// by shape).
static void fine_local_solve(msdd_ctx* c, hipStream_t s, double* u, int variant) {
  FineLevel& F = c->F;
  const bool f32 = c->opt.precision == MSDD_MIXED;
  if (F.twist_built && variant == 3) {
    const bool ok =
        f32 ? launch_apply_fine_twist(s, F.P, F.nd_max, F.bd_max, F.nd.p, F.bd.p, F.doff.p,
                                      F.dboff.p, F.LDc32.p, F.LDr32.p, F.tnbt.p, F.tnbb.p,
                                      F.toff.p, F.TGc32.p, F.TGr32.p, F.coff.p, F.TCinv32.p, 1,
                                      F.dscale.p, u)
            : launch_apply_fine_twist(s, F.P, F.nd_max, F.bd_max, F.nd.p, F.bd.p, F.doff.p,
                                      F.dboff.p, F.LDc.p, F.LDr.p, F.tnbt.p, F.tnbb.p, F.toff.p,
                                      F.TGc.p, F.TGr.p, F.coff.p, F.TCinv.p, 0, nullptr, u);
    REQUIRE(ok, "two-sided Dirichlet solves planned for a shape that does not fit");
    return;
  }
  const int v = variant == 3 ? 0 : variant;
  if (f32)
    launch_apply_fine_solve(s, F.P, F.nd_max, F.bd_max, F.nd.p, F.bd.p, F.doff.p, F.dboff.p,
                            F.LDc32.p, F.LDr32.p, 1, F.dscale.p, u, v);
  else
    launch_apply_fine_solve(s, F.P, F.nd_max, F.bd_max, F.nd.p, F.bd.p, F.doff.p, F.dboff.p,
                            F.LDc.p, F.LDr.p, 0, nullptr, u, v);
}

// dot_partial (PCG): also the chunk partial sums of r.z, written by the gather kernel
void apply_prec(msdd_ctx* c, const double* r, double* z, hipStream_t s,
                double* dot_partial = nullptr) {
  FineLevel& F = c->F;
  const int L = c->n_levels - 1;
  double* rc_top = c->rlev[L - 1].p;  // level L-1 vector
  const bool fork = !c->prof.on;
  if (fork) ensure_side_stream(c);
  const hipStream_t cs = fork ? c->cstream : s;
  {
    // gather (index + value) and u write, PhiD read, rc write
    ProfScope ps(c, PR_APPLY_RESTRICT, F.s_nd * (4.0 + 8.0 + 8.0) + F.s_ndm * 8.0 + F.s_m * 8.0,
                 2.0 * F.s_ndm);
    launch_apply_fine_restrict(s, F.P, F.nd_max, F.nd.p, F.doff.p, F.dglob.p, F.dm.p, F.moff.p,
                               F.phid_off.p, F.PhiD.p, r, rc_top, c->u.p);
  }
  if (fork) {
    HIPCHK(hipEventRecord(c->cev0, s));
    HIPCHK(hipStreamWaitEvent(cs, c->cev0, 0));
  }
  {
    // both sweeps read the band factor once; u is read and written (and the scaling
    // read twice in single precision)
    const bool f32 = c->opt.precision == MSDD_MIXED;
    ProfScope ps(c, PR_APPLY_FINE,
                 2.0 * F.s_dband * (f32 ? 4.0 : 8.0) + 2.0 * F.s_nd * 8.0 + (f32 ? 2.0 * F.s_nd * 8.0 : 0.0),
                 4.0 * F.s_ndbd + F.s_nd);
    fine_local_solve(c, s, c->u.p, c->tune.fine_solve);
  }
  {
    double acb = 0, acf = 0;
    apply_coarse_work(c, &acb, &acf);
    ProfScope ps(c, PR_APPLY_COARSE, acb, acf);
    // coarse levels, downward: C[t] is level L-1-t
    for (int t = 0; t < (int)c->C.size(); ++t) {
      CoarseLevel& CL = c->C[t];
      const int l = CL.level;
      launch_apply_coarse_down(cs, CL.P, CL.no_max, CL.dno.p, CL.own_ptr.p, CL.own_idx.p,
                               CL.loff.p, CL.Inv.p, CL.dm.p, CL.yoff.p, CL.Y.p, CL.moff.p,
                               c->rlev[l].p, c->zlev[l].p, c->rlev[l - 1].p);
    }
    launch_apply_coarsest(cs, c->n0_blocks, c->n0_max, c->z0off.p, c->a0off.p, c->n0blk.p,
                          c->A0inv.p, c->rlev[0].p, c->zlev[0].p);
    for (int t = (int)c->C.size() - 1; t >= 0; --t) {
      CoarseLevel& CL = c->C[t];
      const int l = CL.level;
      launch_apply_coarse_up(cs, CL.P, CL.dno.p, CL.own_ptr.p, CL.own_idx.p, CL.dm.p, CL.yoff.p,
                             CL.Y.p, CL.moff.p, c->zlev[l - 1].p, c->zlev[l].p);
    }
  }
  if (fork) {
    HIPCHK(hipEventRecord(c->cev1, cs));
    HIPCHK(hipStreamWaitEvent(s, c->cev1, 0));
  }
  {
    // with the r.z partial sums: r read as well
    ProfScope ps(c, PR_APPLY_GATHER,
                 (double)(c->n + 1) * 8.0 + F.s_nd * 16.0 + F.s_ndm * 8.0 + c->n * 8.0 + F.s_m * 8.0 +
                     (dot_partial ? c->n * 8.0 : 0.0),
                 2.0 * F.s_ndm + F.s_nd + (dot_partial ? 2.0 * c->n : 0.0));
    if (dot_partial)
      launch_apply_fine_up_dot(s, c->nch, c->ch_lo.p, c->ch_hi.p, F.dinc_ptr.p, F.dinc_sub.p,
                               F.dinc_q.p, F.doff.p, F.dm.p, F.moff.p, F.phid_off.p, F.PhiD.p,
                               c->u.p, c->zlev[L - 1].p, z, r, dot_partial);
    else
      launch_apply_fine_up(s, c->n, F.dinc_ptr.p, F.dinc_sub.p, F.dinc_q.p, F.doff.p, F.dm.p,
                           F.moff.p, F.phid_off.p, F.PhiD.p, c->u.p, c->zlev[L - 1].p, z);
  }
}

// Hybrid form (Sec. 2.1; the form used with GMRES in Sec. 5): restricted additive Schwarz
// on the finest level (local solutions weighted by the partition of unity), then, finest to
// coarsest, each level's additive correction of the updated residual:
//   z = sum_i R_i^T D_i A_i^{-1} R_i r;   for l = L-1, ..., 0:  z += P_l B_l P_l^T (r - A z)
// (B_l: the owned blocks' inverses, level 0 the coarsest inverse).  On one stream.
void apply_hybrid(msdd_ctx* c, const double* r, double* z, hipStream_t s) {
  FineLevel& F = c->F;
  const int L = c->n_levels - 1;
  const int64_t n = c->n;
  double* rc_top = c->rlev[L - 1].p;
  const bool f32 = c->opt.precision == MSDD_MIXED;
  auto fine_restrict = [&](const double* v) {
    ProfScope ps(c, PR_APPLY_RESTRICT, F.s_nd * (4.0 + 8.0 + 8.0) + F.s_ndm * 8.0 + F.s_m * 8.0,
                 2.0 * F.s_ndm);
    launch_apply_fine_restrict(s, F.P, F.nd_max, F.nd.p, F.doff.p, F.dglob.p, F.dm.p, F.moff.p,
                               F.phid_off.p, F.PhiD.p, v, rc_top, c->u.p);
  };
  fine_restrict(r);
  {
    ProfScope ps(c, PR_APPLY_FINE,
                 2.0 * F.s_dband * (f32 ? 4.0 : 8.0) + 2.0 * F.s_nd * 8.0 + (f32 ? 2.0 * F.s_nd * 8.0 : 0.0),
                 4.0 * F.s_ndbd + F.s_nd);
    fine_local_solve(c, s, c->u.p, c->tune.fine_solve);
  }
  {
    ProfScope ps(c, PR_APPLY_GATHER, (double)(n + 1) * 8.0 + F.s_nd * 24.0 + n * 8.0, 2.0 * F.s_nd);
    launch_apply_fine_up(s, n, F.dinc_ptr.p, F.dinc_sub.p, F.dinc_q.p, F.doff.p, F.dm.p, F.moff.p,
                         F.phid_off.p, F.PhiD.p, c->u.p, nullptr, z, F.dw.p, 0);
  }
  double* t = c->hyb_t.p;
  double* q = c->hyb_q.p;
  for (int l = L - 1; l >= 0; --l) {
    {
      ProfScope ps(c, PR_SPMV, (double)c->nnz * 12.0 + (double)(n + 1) * 8.0 + 3.0 * n * 8.0,
                   2.0 * c->nnz);
      launch_spmv_chunk(s, c->nch, c->spmv_sg, c->ch_lo.p, c->ch_hi.p, c->rowptr.p, c->col.p,
                        c->val.p, z, q, c->partial.p);
      launch_residual_chunk(s, c->nch, c->ch_lo.p, c->ch_hi.p, r, q, t, c->partial.p);
    }
    fine_restrict(t);  // rc_top = P_{L-1}^T t (the local copies in u are not used)
    double acb = 0, acf = 0;
    apply_coarse_work(c, &acb, &acf);
    ProfScope ps(c, PR_APPLY_COARSE, acb, acf);
    // restriction down to level l (owned solves of the levels passed are not used), then the
    // solve on level l
    for (int tt = 0; tt < (int)c->C.size(); ++tt) {
      CoarseLevel& CL = c->C[tt];
      const int lv = CL.level;
      if (lv < l) break;
      launch_apply_coarse_down(s, CL.P, CL.no_max, CL.dno.p, CL.own_ptr.p, CL.own_idx.p,
                               CL.loff.p, CL.Inv.p, CL.dm.p, CL.yoff.p, CL.Y.p, CL.moff.p,
                               c->rlev[lv].p, c->zlev[lv].p, c->rlev[lv - 1].p);
    }
    if (l == 0)
      launch_apply_coarsest(s, c->n0_blocks, c->n0_max, c->z0off.p, c->a0off.p, c->n0blk.p,
                            c->A0inv.p, c->rlev[0].p, c->zlev[0].p);
    // prolongation of the level-l correction alone up to level L-1, then to the fine level
    for (int lv = l + 1; lv <= L - 1; ++lv) launch_fill(s, c->nlev[lv], 0.0, c->zlev[lv].p);
    for (int tt = (int)c->C.size() - 1; tt >= 0; --tt) {
      CoarseLevel& CL = c->C[tt];
      const int lv = CL.level;
      if (lv <= l) continue;
      launch_apply_coarse_up(s, CL.P, CL.dno.p, CL.own_ptr.p, CL.own_idx.p, CL.dm.p, CL.yoff.p,
                             CL.Y.p, CL.moff.p, c->zlev[lv - 1].p, c->zlev[lv].p);
    }
    launch_apply_fine_up(s, n, F.dinc_ptr.p, F.dinc_sub.p, F.dinc_q.p, F.doff.p, F.dm.p, F.moff.p,
                         F.phid_off.p, F.PhiD.p, nullptr, c->zlev[L - 1].p, z, nullptr, 1);
  }
}



}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void msdd_default_options(msdd_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = MSDD_FP64;
  o->sigma = 0.0;
  o->eps_reg_rel = 1e-12;
  o->nev_max = 0;
  o->eig_tol = 1e-14;
  o->eig_maxit = 200;
  o->block = 16;
  o->device = 0;
  o->stream = nullptr;
  o->verbose = 0;
  o->geneo_rhs = 1;
  o->nev_fixed = 0;
  o->eig_tol_energy = 1e-10;
  o->dirichlet_rule = 0;
  o->eig_fp32 = 0;
}

int msdd_create(msdd_ctx** out, const msdd_options* opt) {
  if (!out) return MSDD_EINVAL;
  *out = nullptr;
  msdd_ctx* c = new (std::nothrow) msdd_ctx();
  if (!c) return MSDD_ENOMEM;
  if (opt) c->opt = *opt;
  else msdd_default_options(&c->opt);
  std::memset(&c->stats, 0, sizeof(c->stats));
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    delete c;
    return MSDD_EDEVICE;
  }
  if (c->opt.device < 0 || c->opt.device >= ndev || hipSetDevice(c->opt.device) != hipSuccess) {
    delete c;
    return MSDD_EDEVICE;
  }
  if ((c->opt.precision != MSDD_FP64 && c->opt.precision != MSDD_MIXED) ||
      c->opt.geneo_rhs < 1 || c->opt.geneo_rhs > 3 || c->opt.nev_fixed < 0 ||
      (c->opt.dirichlet_rule != 0 && c->opt.dirichlet_rule != 1) ||
      (c->opt.eig_fp32 != 0 && c->opt.eig_fp32 != 1) ||
      (c->opt.eig_fp32 == 1 && c->opt.geneo_rhs != 1)) {
    delete c;
    return MSDD_EINVAL;
  }
  c->stream = (hipStream_t)c->opt.stream;
  // device address of msdd_solve_noalloc's scratch array on this device (once per device)
  if (noalloc_scratch_init(c->opt.device) != 0) {
    delete c;
    return MSDD_EDEVICE;
  }
  *out = c;
  return MSDD_OK;
}

namespace {
int setup_impl(msdd_ctx* c, int64_t n, const int64_t* rowptr, const int32_t* col,
               const double* val, int32_t n_elem, int32_t k, const int32_t* elem_dofs,
               const double* elem_mat, int32_t n_sub, const int64_t* sub_elem_ptr,
               const int32_t* sub_elem, const int64_t* sub_dof_ptr, const int32_t* sub_dof,
               const double* sub_pou, int32_t n_levels, const int32_t* parent, double eta,
               int32_t nprob, const int64_t* prob_dof_ptr) {
  if (!c) return MSDD_EINVAL;
  c->ready = false;
  c->err.clear();
  try {
    REQUIRE(nprob >= 1, "nprob must be positive");
    HIPCHK(hipSetDevice(c->opt.device));
    DevicePool::get().safe_point();  // the previous setup's freed buffers become reusable
    const double t0 = now_ms();
    REQUIRE(n > 0 && n < (int64_t)1 << 31, "n out of range");
    REQUIRE(n_elem > 0 && k > 0 && k <= 81, "bad element count or size");
    REQUIRE(n_sub > 0, "n_sub must be positive");
    REQUIRE(n_levels >= 2 && n_levels <= 8, "n_levels must be in [2, 8]");
    REQUIRE(eta > 0 && std::isfinite(eta), "eta must be positive");
    REQUIRE(c->opt.eig_maxit > 0 && c->opt.eig_tol > 0 && c->opt.eig_tol_energy >= 0,
            "bad eigensolver options");
    REQUIRE(c->opt.dirichlet_rule == 0 || c->opt.dirichlet_rule == 1,
            "dirichlet_rule must be 0 or 1");
    REQUIRE(c->opt.eig_fp32 == 0 || (c->opt.eig_fp32 == 1 && c->opt.geneo_rhs == 1),
            "eig_fp32 must be 0, or 1 with geneo_rhs = 1");
    c->n = n;
    c->k = k;
    c->eta = eta;
    c->sigma = c->opt.sigma > 0 ? c->opt.sigma : 0.1 * eta;
    c->n_levels = n_levels;
    hipStream_t s = c->stream;
    double tv = now_ms();
    // host copies of the index arrays (planning)
    std::vector<int64_t>& h_rowptr = c->in_rowptr;
    to_host_into(h_rowptr, rowptr, (size_t)n + 1);
    REQUIRE(h_rowptr[0] == 0, "rowptr[0] must be 0");
    {
      const int nr = host_threads((int)std::min<int64_t>(16, (n + 65535) / 65536));
      std::vector<int64_t> first(nr, -1);
      parallel_for(nr, nr, [&](int t, int) {
        for (int64_t i = n * t / nr; i < n * (t + 1) / nr; ++i)
          if (h_rowptr[i + 1] < h_rowptr[i]) {
            first[t] = i;
            break;
          }
      });
      for (int t = 0; t < nr; ++t) REQUIRE(first[t] < 0, "rowptr not monotone");
    }
    c->nnz = h_rowptr[n];
    std::vector<int32_t>& ed = c->in_ed;
    std::vector<int64_t>& sep = c->in_sep;
    std::vector<int64_t>& sdp = c->in_sdp;
    to_host_into(sep, sub_elem_ptr, (size_t)n_sub + 1);
    to_host_into(sdp, sub_dof_ptr, (size_t)n_sub + 1);
    REQUIRE(sep[0] == 0 && sdp[0] == 0, "subdomain pointers must start at 0");
    std::vector<int32_t>& se = c->in_se;
    std::vector<int32_t>& sd = c->in_sd;
    std::vector<double>& sw = c->in_sw;
    {
      // the element and subdomain arrays: device sources of up to 16 MB leave together as
      // asynchronous copies on the null stream (ordered as the synchronous copies are
      // against the caller's work) into pinned staging, then move to the host vectors in
      // parallel; larger or host sources go one by one
      struct In {
        void* dst;
        const void* src;
        size_t bytes;
        char* st;
      };
      std::vector<In> batch;
      auto take = [&](auto& v, const auto* src, size_t cnt) {
        v.resize(cnt);
        const size_t bytes = cnt * sizeof(v[0]);
        char* st = nullptr;
        if (cnt && src && is_device_ptr(src) && bytes <= ((size_t)16 << 20))
          st = static_cast<char*>(PinnedArena::get().alloc(bytes));
        if (st)
          batch.push_back({v.data(), src, bytes, st});
        else
          to_host_into(v, src, cnt);
      };
      take(ed, elem_dofs, (size_t)n_elem * k);
      take(se, sub_elem, (size_t)sep[n_sub]);
      take(sd, sub_dof, (size_t)sdp[n_sub]);
      take(sw, sub_pou, (size_t)sdp[n_sub]);
      for (const In& b : batch)
        HIPCHK(hipMemcpyAsync(b.st, b.src, b.bytes, hipMemcpyDeviceToHost, nullptr));
      HIPCHK(hipStreamSynchronize(nullptr));
      // out of staging in pieces of 1 MB over the planning threads
      constexpr size_t kPc = (size_t)1 << 20;
      std::vector<std::pair<int, size_t>> pieces;
      for (int q = 0; q < (int)batch.size(); ++q)
        for (size_t a = 0; a < batch[q].bytes; a += kPc) pieces.push_back({q, a});
      parallel_for((int)pieces.size(), host_threads((int)pieces.size()), [&](int t, int) {
        const In& b = batch[pieces[t].first];
        const size_t a = pieces[t].second, len = std::min(kPc, b.bytes - a);
        std::memcpy(static_cast<char*>(b.dst) + a, b.st + a, len);
      });
    }
    vlog(c, "setup: host copies of the index inputs", &tv);
    std::vector<std::vector<int32_t>> parents;
    {
      int cnt = n_sub;
      size_t off = 0;
      std::vector<int32_t> all;
      for (int l = 0; l < n_levels - 2; ++l) {
        std::vector<int32_t> pm = to_host(parent + off, (size_t)cnt);
        int mx = -1;
        for (int32_t v : pm) {
          REQUIRE(v >= 0 && v < cnt, "parent index out of range");
          mx = std::max(mx, v);
        }
        parents.push_back(pm);
        off += cnt;
        cnt = mx + 1;
      }
    }
    // problems of a batch: dof ranges; every subdomain lies in one problem, subdomains
    // are ordered by problem on every level, and A does not couple problems
    std::vector<int64_t> pdp = prob_dof_ptr ? to_host(prob_dof_ptr, (size_t)nprob + 1)
                                            : std::vector<int64_t>{0, n};
    REQUIRE(pdp[0] == 0 && pdp[nprob] == n, "problem dof pointers must run from 0 to n");
    for (int t = 0; t < nprob; ++t) REQUIRE(pdp[t + 1] > pdp[t], "empty problem in the batch");
    std::vector<int32_t> prob_cur(n_sub, 0);
    if (nprob > 1) {
      for (int i = 0; i < n_sub; ++i) {
        REQUIRE(sdp[i + 1] > sdp[i], "subdomain without dofs in a batch");
        const int32_t d0 = sd[sdp[i]];
        REQUIRE(d0 >= 0 && d0 < n, "sub_dof entry out of range");
        const int t = (int)(std::upper_bound(pdp.begin(), pdp.end(), (int64_t)d0) - pdp.begin()) - 1;
        for (int64_t q = sdp[i]; q < sdp[i + 1]; ++q)
          REQUIRE(sd[q] >= pdp[t] && sd[q] < pdp[t + 1],
                  "subdomain " + std::to_string(i) + " spans two problems");
        prob_cur[i] = t;
        REQUIRE(i == 0 || t >= prob_cur[i - 1], "subdomains must be ordered by problem");
      }
      std::vector<char> has(nprob, 0);
      for (int32_t t : prob_cur) has[t] = 1;
      for (int t = 0; t < nprob; ++t) REQUIRE(has[t], "problem " + std::to_string(t) + " has no subdomain");
    }
    std::vector<std::vector<int32_t>> prob_lvl(1, prob_cur);  // [0] = finest, then coarser
    for (const auto& pm : parents) {
      const auto& pf = prob_lvl.back();
      int cnt = 0;
      for (int32_t v : pm) cnt = std::max(cnt, v + 1);
      std::vector<int32_t> pc(cnt, -1);
      for (size_t j = 0; j < pm.size(); ++j) {
        REQUIRE(pc[pm[j]] < 0 || pc[pm[j]] == pf[j], "a coarse subdomain spans two problems");
        pc[pm[j]] = pf[j];
      }
      for (int i = 0; i < cnt; ++i) {
        REQUIRE(pc[i] >= 0, "coarse subdomain " + std::to_string(i) + " has no children");
        REQUIRE(i == 0 || pc[i] >= pc[i - 1], "coarse subdomains must be ordered by problem");
      }
      prob_lvl.push_back(pc);
    }
    c->nseg = nprob;
    c->h_seg_row = pdp;
    // device copies kept by the context
    to_device(c->rowptr, rowptr, (size_t)n + 1, s);
    to_device(c->col, col, (size_t)c->nnz, s);
    to_device(c->val, val, (size_t)c->nnz, s);
    if (nprob > 1) {
      // A must not couple problems: checked on the device copies, one thread per row
      DVec<int64_t> dpdp;
      dpdp.upload(pdp, s);
      DVec<int> flag;
      flag.alloc(1);
      flag.zero(s);
      launch_check_problem_coupling(s, n, c->rowptr.p, c->col.p, dpdp.p, nprob, flag.p);
      HIPCHK(hipGetLastError());
      REQUIRE(flag.download(s)[0] == 0, "the matrix couples two problems");
    }
    DVec<double> emat_holder;
    const double* d_emat = elem_mat;
    if (!is_device_ptr(elem_mat)) {
      to_device(emat_holder, elem_mat, (size_t)n_elem * k * k, s);
      d_emat = emat_holder.p;
    }
    vlog(c, "setup: input copies", &tv);
    const double avg = (double)c->nnz / (double)n;
    c->spmv_sg = c->tune.spmv_group > 0 ? c->tune.spmv_group
                                        : (avg <= 6 ? 4 : (avg <= 14 ? 8 : (avg <= 40 ? 16 : 32)));
    // finest level
    c->F = FineLevel();
    c->F.P = n_sub;
    const std::vector<int32_t>* wp = nullptr;
    if (c->warm.P > 0) {
      REQUIRE(c->warm.P == n_sub, "warm start attached for " + std::to_string(c->warm.P) +
                                      " subdomains, setup has " + std::to_string(n_sub));
      REQUIRE(c->warm.n_entries == sdp[n_sub], "warm start frame positions do not match sub_dof");
      if (c->warm.net)
        REQUIRE(msdd_net_internal::device(c->warm.net) == c->opt.device,
                "warm-start network lives on another device");
      wp = &c->warm.pos;
    }
    c->warm.have_targets = false;
    plan_fine(c, n_elem, ed, sep, se, sdp, sd, sw, wp);
    {
      std::vector<int32_t> sid(n_sub);
      for (int i = 0, first = 0; i < n_sub; ++i) {
        if (i > 0 && prob_cur[i] != prob_cur[i - 1]) first = i;
        sid[i] = i - first;
      }
      c->F.seed_id.upload(sid, s);
    }
    const double t1 = now_ms();  // host planning done; its uploads may still be in flight
    // the symbolic planning of the finest-level patches runs on a host thread (uploads on
    // a side stream) while the GPU factorises and solves the local eigenproblems
    if (!c->ustream) HIPCHK(hipStreamCreateWithFlags(&c->ustream, hipStreamNonBlocking));
    PatchLevel PL;
    PatchPlan PT;
    MsddError plan_err{MSDD_OK, ""};
    std::thread plan_thread([&] {
      try {
        HIPCHK(hipSetDevice(c->opt.device));
        fine_patches_plan(c, ed, n_elem, PL, PT, c->ustream);
        HIPCHK(hipStreamSynchronize(c->ustream));
      } catch (const MsddError& e) {
        plan_err = e;
      }
    });
    struct Joiner {
      std::thread& t;
      ~Joiner() {
        if (t.joinable()) t.join();
      }
    } joiner{plan_thread};
    fine_local_matrices(c, d_emat);
    HIPCHK(hipStreamSynchronize(s));
    const double t2 = now_ms();
    fine_eigensolve(c);
    HIPCHK(hipStreamSynchronize(s));
    const double t3 = now_ms();
    plan_thread.join();
    if (plan_err.code != MSDD_OK) throw plan_err;
    // coarse levels
    const int L = n_levels - 1;
    c->C.clear();
    c->C.resize(L - 1);
    fine_patches(c, d_emat, PL, PT);
    std::vector<int32_t> m_cur = c->F.m;
    std::vector<int64_t> moff_cur = c->F.h_moff;
    for (int t = 0; t < L - 1; ++t) {
      const int l = L - 1 - t;
      PatchLevel PLn;
      coarse_level(c, l, parents[t], m_cur, moff_cur, PL, c->C[t], PLn);
      PL = std::move(PLn);
      m_cur = c->C[t].m;
      moff_cur = c->C[t].h_moff;
    }
    coarsest(c, PL, m_cur, prob_lvl.back(), nprob);
    HIPCHK(hipStreamSynchronize(s));
    const double t4 = now_ms();
    // level sizes
    c->nlev.assign(L + 1, 0);
    c->nlev[L] = n;
    c->nlev[L - 1] = c->F.h_moff.back();
    for (int t = 0; t < L - 1; ++t) c->nlev[L - 2 - t] = c->C[t].h_moff.back();
    alloc_solve_work(c);
    HIPCHK(hipStreamSynchronize(s));
    const double t5 = now_ms();
    msdd_stats_t& st = c->stats;
    st.n_levels = n_levels;
    for (int l = 0; l <= L && l < 8; ++l) st.n[l] = c->nlev[l];
    st.n_sub[L] = n_sub;
    st.n_sub[0] = nprob;
    int mm = 0;
    for (int v : c->F.m) mm = std::max(mm, v);
    st.m_max[L] = mm;
    st.max_local[L] = c->F.nb_max;
    for (int t = 0; t < L - 1; ++t) {
      const int l = L - 1 - t;
      st.n_sub[l] = c->C[t].P;
      int m2 = 0, g2 = 0;
      for (int v : c->C[t].m) m2 = std::max(m2, v);
      for (int v : c->C[t].ng) g2 = std::max(g2, v);
      st.m_max[l] = m2;
      st.max_local[l] = g2;
    }
    st.max_band = c->F.bw_max;
    st.t_plan_ms = t1 - t0;
    st.t_local_ms = t2 - t1;
    st.t_gevp_ms = t3 - t2;
    st.t_coarse_ms = t4 - t3;
    st.t_setup_ms = t5 - t0;
    c->ready = true;
    if (c->opt.verbose)
      std::fprintf(stderr, "msdd setup: plan %.2f local %.2f gevp %.2f coarse %.2f total %.2f ms, n0=%d\n",
                   st.t_plan_ms, st.t_local_ms, st.t_gevp_ms, st.t_coarse_ms, st.t_setup_ms, c->n0);
    return MSDD_OK;
  } catch (const MsddError& e) {
    return code_for(c, e);
  } catch (const std::exception& e) {
    return code_for(c, MsddError{MSDD_ENOMEM, e.what()});
  }
}
}  // namespace

int msdd_setup(msdd_ctx* c, int64_t n, const int64_t* rowptr, const int32_t* col,
               const double* val, int32_t n_elem, int32_t k, const int32_t* elem_dofs,
               const double* elem_mat, int32_t n_sub, const int64_t* sub_elem_ptr,
               const int32_t* sub_elem, const int64_t* sub_dof_ptr, const int32_t* sub_dof,
               const double* sub_pou, int32_t n_levels, const int32_t* parent, double eta) {
  return setup_impl(c, n, rowptr, col, val, n_elem, k, elem_dofs, elem_mat, n_sub, sub_elem_ptr,
                    sub_elem, sub_dof_ptr, sub_dof, sub_pou, n_levels, parent, eta, 1, nullptr);
}

int msdd_setup_batch(msdd_ctx* c, int32_t nprob, const int64_t* prob_dof_ptr, int64_t n,
                     const int64_t* rowptr, const int32_t* col, const double* val,
                     int32_t n_elem, int32_t k, const int32_t* elem_dofs,
                     const double* elem_mat, int32_t n_sub, const int64_t* sub_elem_ptr,
                     const int32_t* sub_elem, const int64_t* sub_dof_ptr,
                     const int32_t* sub_dof, const double* sub_pou, int32_t n_levels,
                     const int32_t* parent, double eta) {
  if (!prob_dof_ptr) return c ? code_for(c, MsddError{MSDD_EINVAL, "null prob_dof_ptr"}) : MSDD_EINVAL;
  return setup_impl(c, n, rowptr, col, val, n_elem, k, elem_dofs, elem_mat, n_sub, sub_elem_ptr,
                    sub_elem, sub_dof_ptr, sub_dof, sub_pou, n_levels, parent, eta, nprob,
                    prob_dof_ptr);
}

int msdd_apply(msdd_ctx* c, const double* r, double* z) {
  if (!c) return MSDD_EINVAL;
  if (!c->ready) return code_for(c, MsddError{MSDD_ESTATE, "msdd_apply before a successful setup"});
  try {
    HIPCHK(hipSetDevice(c->opt.device));
    hipStream_t s = c->stream;
    const int64_t n = c->n;
    const bool rdev = is_device_ptr(r), zdev = is_device_ptr(z);
    const double* rin = r;
    if (!rdev) {
      HIPCHK(hipMemcpyAsync(c->r.p, r, n * sizeof(double), hipMemcpyHostToDevice, s));
      rin = c->r.p;
    }
    double* zout = zdev ? z : c->z.p;
    apply_prec(c, rin, zout, s);
    HIPCHK(hipGetLastError());
    if (!zdev) HIPCHK(hipMemcpyAsync(z, zout, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return MSDD_OK;
  } catch (const MsddError& e) {
    return code_for(c, e);
  }
}

namespace {

// Device buffers of one PCG run: work vectors, chunk partial sums, per-segment scalars
// and states, residual history ((maxit + 1) entries per segment).
struct PcgBufs {
  double *r, *z, *p, *q, *partial, *segD, *hist;
  int* segI;
};

PcgBufs ctx_bufs(msdd_ctx* c) {
  return PcgBufs{c->r.p, c->z.p, c->p.p, c->q.p, c->partial.p, c->segD.p, c->hist_d.p, c->segI.p};
}

// One PCG iteration on every segment (Sec. 5), launched on stream s.
void pcg_iteration(msdd_ctx* c, hipStream_t s, double* xx, int maxit, const PcgBufs& w) {
  const int64_t n = c->n;
  const int nch = c->nch, ns = c->nseg;
  const double spmv_bytes = (double)c->nnz * 12.0 + (double)(n + 1) * 8.0 + 2.0 * n * 8.0;
  {
    ProfScope ps(c, PR_SPMV, spmv_bytes, 2.0 * c->nnz);
    launch_spmv_chunk(s, nch, c->spmv_sg, c->ch_lo.p, c->ch_hi.p, c->rowptr.p, c->col.p, c->val.p,
                      w.p, w.q, w.partial);
  }
  {
    ProfScope ps(c, PR_VEC, 6.0 * n * 8.0, 6.0 * n);
    launch_seg_reduce(s, ns, c->seg_ch.p, w.partial, w.segD, w.segI, PCG_R_PQ, 0.0, maxit, w.hist);
    launch_update_xr_chunk(s, nch, c->ch_lo.p, c->ch_hi.p, c->ch_seg.p, xx, w.r, w.p, w.q, w.segD,
                           w.partial);
    launch_seg_reduce(s, ns, c->seg_ch.p, w.partial, w.segD, w.segI, PCG_R_RR, 0.0, maxit, w.hist);
  }
  apply_prec(c, w.r, w.z, s, w.partial);  // z = M r and the chunk sums of r.z
  {
    ProfScope ps(c, PR_VEC, 3.0 * n * 8.0, 2.0 * n);
    launch_seg_reduce(s, ns, c->seg_ch.p, w.partial, w.segD, w.segI, PCG_R_RZ, 0.0, maxit, w.hist);
    launch_update_p_chunk(s, nch, c->ch_lo.p, c->ch_hi.p, c->ch_seg.p, w.z, w.p, w.segD, 0);
  }
}

// Iterations run in chunks of PCG_CHUNK without reading anything back; a segment that
// converged is frozen on the device (alpha = beta = 0).  Without profiling, a chunk is
// captured once as a HIP graph (per x pointer and maxit) and replayed.
constexpr int PCG_CHUNK = 8;

bool any_running(msdd_ctx* c, const PcgBufs& w) {
  HIPCHK(hipMemcpyAsync(c->h_segI, w.segI, (size_t)c->nseg * PCG_SI * sizeof(int),
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int q = 0; q < c->nseg; ++q)
    if (c->h_segI[q * PCG_SI + PCG_ACTIVE] == PCG_RUNNING) return true;
  return false;
}

void run_chunk(msdd_ctx* c, double* xx, const double* bb, int maxit, const PcgBufs& w, bool graph) {
  if (c->prof.on || !graph) {
    for (int k = 0; k < PCG_CHUNK; ++k) pcg_iteration(c, c->stream, xx, maxit, w);
    return;
  }
  if (!c->gstream) {
    HIPCHK(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c->gev0, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->gev1, hipEventDisableTiming));
  }
  if (!c->gexec || c->g_x != xx || c->g_b != bb || c->g_maxit != maxit) {
    if (c->gexec) HIPCHK(hipGraphExecDestroy(c->gexec));
    c->gexec = nullptr;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < PCG_CHUNK; ++k) pcg_iteration(c, c->gstream, xx, maxit, w);
    HIPCHK(hipStreamEndCapture(c->gstream, &g));
    const hipError_t e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
    c->g_x = xx;
    c->g_b = bb;
    c->g_maxit = maxit;
  }
  HIPCHK(hipEventRecord(c->gev0, c->stream));
  HIPCHK(hipStreamWaitEvent(c->gstream, c->gev0, 0));
  HIPCHK(hipGraphLaunch(c->gexec, c->gstream));
  HIPCHK(hipEventRecord(c->gev1, c->gstream));
  HIPCHK(hipStreamWaitEvent(c->stream, c->gev1, 0));
}

// PCG on all segments from the initial guess in xx (device), right-hand side bb (device),
// with the buffers w; per-segment iteration counts and final recurrence residuals in
// c->last_iters / c->last_relres, the history of segment 0 in c->hist.  Returns the status.
int pcg_run(msdd_ctx* c, const double* bb, double* xx, double rtol, int32_t maxit,
            const PcgBufs& w, bool graph, double t0) {
  hipStream_t s = c->stream;
  const int ns = c->nseg;
  // r = b - A x, rr0 per segment
  launch_spmv_chunk(s, c->nch, c->spmv_sg, c->ch_lo.p, c->ch_hi.p, c->rowptr.p, c->col.p, c->val.p,
                    xx, w.q, w.partial);
  launch_residual_chunk(s, c->nch, c->ch_lo.p, c->ch_hi.p, bb, w.q, w.r, w.partial);
  launch_seg_reduce(s, ns, c->seg_ch.p, w.partial, w.segD, w.segI, PCG_R_RR0, rtol, maxit, w.hist);
  apply_prec(c, w.r, w.z, s, w.partial);
  launch_seg_reduce(s, ns, c->seg_ch.p, w.partial, w.segD, w.segI, PCG_R_RZ0, 0.0, maxit, w.hist);
  launch_update_p_chunk(s, c->nch, c->ch_lo.p, c->ch_hi.p, c->ch_seg.p, w.z, w.p, w.segD, 1);
  HIPCHK(hipGetLastError());
  int done_its = 0;
  while (any_running(c, w) && done_its < maxit) {
    run_chunk(c, xx, bb, maxit, w, graph);
    HIPCHK(hipGetLastError());
    done_its += PCG_CHUNK;
  }
  std::vector<double> D((size_t)ns * PCG_SD);
  std::vector<int> I((size_t)ns * PCG_SI);
  HIPCHK(hipMemcpyAsync(D.data(), w.segD, D.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(I.data(), w.segI, I.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  c->last_iters.assign(ns, 0);
  c->last_relres.assign(ns, 0.0);
  int status = MSDD_OK;
  bool bad = false;
  for (int q = 0; q < ns; ++q) {
    const int act = I[q * PCG_SI + PCG_ACTIVE];
    c->last_iters[q] = act == PCG_RUNNING ? I[q * PCG_SI + PCG_IT] : I[q * PCG_SI + PCG_ITERS];
    const double rr0 = D[q * PCG_SD + PCG_RR0];
    c->last_relres[q] = rr0 > 0 ? std::sqrt(D[q * PCG_SD + PCG_RR] / rr0) : 0.0;
    if (act == PCG_BREAKDOWN) bad = true;
    else if (act != PCG_CONVERGED) status = MSDD_ENOCONV;
  }
  REQUIRE(!bad, "PCG produced a non-finite value (breakdown or non-finite input)");
  // residual history of segment 0 (entry k of segment q at k * ns + q)
  const int it0 = c->last_iters[0];
  c->hist.assign(it0 + 1, 0.0);
  HIPCHK(hipMemcpy2DAsync(c->hist.data(), sizeof(double), w.hist, (size_t)ns * sizeof(double),
                          sizeof(double), (size_t)it0 + 1, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  c->stats.pcg_iters = *std::max_element(c->last_iters.begin(), c->last_iters.end());
  c->stats.pcg_relres = *std::max_element(c->last_relres.begin(), c->last_relres.end());
  c->stats.t_solve_ms = now_ms() - t0;
  return status;
}

int solve_all(msdd_ctx* c, const double* b, double* x, double rtol, int32_t maxit) {
  HIPCHK(hipSetDevice(c->opt.device));
  REQUIRE(b && x && rtol > 0 && maxit >= 0, "bad solve arguments");
  hipStream_t s = c->stream;
  const double t0 = now_ms();
  const int64_t n = c->n;
  const int ns = c->nseg;
  const bool bdev = is_device_ptr(b), xdev = is_device_ptr(x);
  const double* bb = b;
  if (!bdev) {
    HIPCHK(hipMemcpyAsync(c->bvec.p, b, n * sizeof(double), hipMemcpyHostToDevice, s));
    bb = c->bvec.p;
  }
  double* xx = xdev ? x : c->x.p;
  if (!xdev) HIPCHK(hipMemcpyAsync(xx, x, n * sizeof(double), hipMemcpyHostToDevice, s));
  // the history holds (maxit + 1) entries per segment; a later setup may have more segments
  if (c->hist_cap < (size_t)(maxit + 1) * ns) {
    c->hist_d.alloc((size_t)(maxit + 1) * ns);
    c->hist_cap = (size_t)(maxit + 1) * ns;
    if (c->gexec) HIPCHK(hipGraphExecDestroy(c->gexec));
    c->gexec = nullptr;
  }
  const int status = pcg_run(c, bb, xx, rtol, maxit, ctx_bufs(c), true, t0);
  if (!xdev) {
    HIPCHK(hipMemcpyAsync(x, xx, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return status;
}

// Restarted GMRES with the hybrid form as right preconditioner (Sec. 5): Arnoldi by
// classical Gram-Schmidt applied twice (the projections of a step in two passes over the
// basis), the Hessenberg least-squares problem by Givens rotations on the host (one small
// read-back per iteration), x = x0 + M V y at the end of a cycle, then b - A x recomputed.
// A cycle ends when its least-squares residual meets rtol ||r_0|| or after `restart` steps.
// The solve stops when the recomputed residual meets the tolerance; after a cycle that met
// it only in the least-squares sense the next cycle refines from x, unless that cycle
// reduced the recomputed residual by less than half: it then sits at its FP64 rounding
// floor (about u || |A| |x| + |b| ||) and the solve stops as converged.
int gmres_run(msdd_ctx* c, const double* bb, double* xx, double rtol, int restart, int maxit) {
  hipStream_t s = c->stream;
  const double t0 = now_ms();
  const int64_t n = c->n;
  const int mr = std::max(1, std::min(restart, std::max(maxit, 1)));
  DVec<double> V, w, zt, hd, part;
  V.alloc((size_t)(mr + 1) * n);
  w.alloc(n);
  zt.alloc(n);
  hd.alloc((size_t)2 * (mr + 2));
  part.alloc((size_t)multi_dot_blocks(n) * (mr + 1));
  double* r = c->r.p;
  auto true_residual = [&]() {  // r = b - A x; returns ||r||
    launch_spmv_chunk(s, c->nch, c->spmv_sg, c->ch_lo.p, c->ch_hi.p, c->rowptr.p, c->col.p,
                      c->val.p, xx, c->q.p, c->partial.p);
    launch_residual_chunk(s, c->nch, c->ch_lo.p, c->ch_hi.p, bb, c->q.p, r, c->partial.p);
    launch_multi_dot(s, n, 1, r, r, part.p, hd.p);
    double rr = 0.0;
    HIPCHK(hipMemcpyAsync(&rr, hd.p, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return std::sqrt(rr);
  };
  double beta = true_residual();
  REQUIRE(std::isfinite(beta), "non-finite right-hand side or initial guess");
  const double r0 = beta;
  c->hist.assign(1, r0 > 0 ? 1.0 : 0.0);
  int its = 0;
  int status = MSDD_ENOCONV;
  if (r0 == 0.0) status = MSDD_OK;
  std::vector<double> H((size_t)(mr + 1) * mr), cs(mr), sn(mr), g(mr + 1), hv(2 * (mr + 2));
  while (status != MSDD_OK && its < maxit) {
    const double beta_start = beta;
    const int m = std::min(mr, maxit - its);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    // v_0 = r / beta (beta^2 is still in hd[0])
    launch_scale_dev(s, n, hd.p, 2, r, V.p);
    int k_done = 0;
    bool conv = false;
    for (int k = 0; k < m; ++k) {
      double* vk = V.p + (size_t)k * n;
      apply_hybrid(c, vk, zt.p, s);
      launch_spmv_chunk(s, c->nch, c->spmv_sg, c->ch_lo.p, c->ch_hi.p, c->rowptr.p, c->col.p,
                        c->val.p, zt.p, w.p, c->partial.p);
      // two passes of classical Gram-Schmidt, then the norm
      launch_multi_dot(s, n, k + 1, V.p, w.p, part.p, hd.p);
      launch_multi_axpy(s, n, k + 1, V.p, hd.p, w.p);
      launch_multi_dot(s, n, k + 1, V.p, w.p, part.p, hd.p + (mr + 2));
      launch_multi_axpy(s, n, k + 1, V.p, hd.p + (mr + 2), w.p);
      launch_multi_dot(s, n, 1, w.p, w.p, part.p, hd.p + (mr + 1));
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(hv.data(), hd.p, hv.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double* Hk = &H[(size_t)k * (mr + 1)];  // column k
      for (int j = 0; j <= k; ++j) Hk[j] = hv[j] + hv[(mr + 2) + j];
      const double hn = std::sqrt(std::max(hv[mr + 1], 0.0));
      REQUIRE(std::isfinite(hn), "GMRES produced a non-finite value");
      Hk[k + 1] = hn;
      if (hn > 0.0) launch_scale_dev(s, n, hd.p + (mr + 1), 2, w.p, V.p + (size_t)(k + 1) * n);
      for (int j = 0; j < k; ++j) {  // earlier rotations on the new column
        const double a = cs[j] * Hk[j] + sn[j] * Hk[j + 1];
        Hk[j + 1] = -sn[j] * Hk[j] + cs[j] * Hk[j + 1];
        Hk[j] = a;
      }
      const double d = std::hypot(Hk[k], Hk[k + 1]);
      cs[k] = Hk[k] / d;
      sn[k] = Hk[k + 1] / d;
      Hk[k] = d;
      Hk[k + 1] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      ++its;
      k_done = k + 1;
      c->hist.push_back(std::fabs(g[k + 1]) / r0);
      if (std::fabs(g[k + 1]) < rtol * r0 || hn == 0.0) {
        conv = std::fabs(g[k + 1]) < rtol * r0;
        break;
      }
    }
    // y = R^{-1} g (upper triangular, column-major in H with ld mr + 1), x += M V y
    std::vector<double> y(k_done);
    for (int i = k_done - 1; i >= 0; --i) {
      double t = g[i];
      for (int j = i + 1; j < k_done; ++j) t -= H[(size_t)j * (mr + 1) + i] * y[j];
      y[i] = t / H[(size_t)i * (mr + 1) + i];
    }
    HIPCHK(hipMemcpyAsync(hd.p, y.data(), k_done * sizeof(double), hipMemcpyHostToDevice, s));
    launch_gemv_cols(s, n, k_done, V.p, hd.p, w.p, 0);
    apply_hybrid(c, w.p, zt.p, s);
    launch_axpy(s, n, 1.0, zt.p, xx);
    beta = true_residual();
    REQUIRE(std::isfinite(beta), "GMRES produced a non-finite value");
    if (beta < rtol * r0 || (conv && beta >= 0.5 * beta_start)) status = MSDD_OK;
  }
  c->last_iters.assign(1, its);
  c->last_relres.assign(1, r0 > 0 ? beta / r0 : 0.0);
  c->stats.pcg_iters = its;
  c->stats.pcg_relres = r0 > 0 ? beta / r0 : 0.0;
  c->stats.t_solve_ms = now_ms() - t0;
  return status;
}

}  // namespace

int msdd_apply_hybrid(msdd_ctx* c, const double* r, double* z) {
  if (!c) return MSDD_EINVAL;
  if (!c->ready) return code_for(c, MsddError{MSDD_ESTATE, "msdd_apply_hybrid before a successful setup"});
  try {
    HIPCHK(hipSetDevice(c->opt.device));
    REQUIRE(c->nseg == 1, "the hybrid form is available for single-problem setups");
    hipStream_t s = c->stream;
    const int64_t n = c->n;
    const bool rdev = is_device_ptr(r), zdev = is_device_ptr(z);
    const double* rin = r;
    if (!rdev) {
      HIPCHK(hipMemcpyAsync(c->bvec.p, r, n * sizeof(double), hipMemcpyHostToDevice, s));
      rin = c->bvec.p;
    }
    double* zout = zdev ? z : c->z.p;
    apply_hybrid(c, rin, zout, s);
    HIPCHK(hipGetLastError());
    if (!zdev) HIPCHK(hipMemcpyAsync(z, zout, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return MSDD_OK;
  } catch (const MsddError& e) {
    return code_for(c, e);
  }
}

int msdd_solve_gmres(msdd_ctx* c, const double* b, double* x, double rtol, int32_t restart,
                     int32_t maxit, int32_t* iters, double* relres) {
  if (!c) return MSDD_EINVAL;
  if (!c->ready) return code_for(c, MsddError{MSDD_ESTATE, "msdd_solve_gmres before a successful setup"});
  try {
    HIPCHK(hipSetDevice(c->opt.device));
    REQUIRE(b && x && rtol > 0 && maxit >= 0 && restart >= 1, "bad solve arguments");
    REQUIRE(c->nseg == 1, "GMRES with the hybrid form is available for single-problem setups");
    hipStream_t s = c->stream;
    const int64_t n = c->n;
    const bool bdev = is_device_ptr(b), xdev = is_device_ptr(x);
    const double* bb = b;
    if (!bdev) {
      HIPCHK(hipMemcpyAsync(c->bvec.p, b, n * sizeof(double), hipMemcpyHostToDevice, s));
      bb = c->bvec.p;
    }
    double* xx = xdev ? x : c->x.p;
    if (!xdev) HIPCHK(hipMemcpyAsync(xx, x, n * sizeof(double), hipMemcpyHostToDevice, s));
    const int st = gmres_run(c, bb, xx, rtol, restart, maxit);
    if (!xdev) {
      HIPCHK(hipMemcpyAsync(x, xx, n * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    if (iters) *iters = c->stats.pcg_iters;
    if (relres) *relres = c->stats.pcg_relres;
    if (st == MSDD_ENOCONV) return code_for(c, MsddError{MSDD_ENOCONV, "GMRES reached maxit"});
    return st;
  } catch (const MsddError& e) {
    return code_for(c, e);
  }
}

int msdd_solve_noalloc(msdd_ctx* c, const double* b, double* x, double rtol, int32_t maxit,
                       int32_t* iters, double* relres) {
  if (!c) return MSDD_EINVAL;
  if (!c->ready)
    return code_for(c, MsddError{MSDD_ESTATE, "msdd_solve_noalloc before a successful setup"});
  try {
    HIPCHK(hipSetDevice(c->opt.device));
    REQUIRE(b && x && rtol > 0 && maxit >= 0, "bad solve arguments");
    REQUIRE(is_device_ptr(b) && is_device_ptr(x), "msdd_solve_noalloc needs device pointers for b and x");
    const double t0 = now_ms();
    const int64_t n = c->n;
    const int ns = c->nseg;
    // carve the buffers from the device's scratch array, each 256-byte aligned
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t b_vec = up((size_t)n * sizeof(double));
    const size_t b_part = up((size_t)std::max(c->nch, 1) * sizeof(double));
    const size_t b_sd = up((size_t)ns * PCG_SD * sizeof(double));
    const size_t b_hist = up((size_t)(maxit + 1) * ns * sizeof(double));
    const size_t b_si = up((size_t)ns * PCG_SI * sizeof(int));
    const size_t need = 4 * b_vec + b_part + b_sd + b_hist + b_si;
    if (need > MSDD_NOALLOC_SCRATCH_BYTES)
      throw MsddError{MSDD_EINVAL, "msdd_solve_noalloc: needs " + std::to_string(need) +
                                       " bytes of scratch, the limit is " +
                                       std::to_string((size_t)MSDD_NOALLOC_SCRATCH_BYTES)};
    unsigned char* base = static_cast<unsigned char*>(noalloc_scratch(c->opt.device));
    REQUIRE(base, "scratch memory of this device not initialised");
    PcgBufs w;
    size_t off = 0;
    auto take = [&](size_t bytes) { unsigned char* q = base + off; off += bytes; return q; };
    w.r = reinterpret_cast<double*>(take(b_vec));
    w.z = reinterpret_cast<double*>(take(b_vec));
    w.p = reinterpret_cast<double*>(take(b_vec));
    w.q = reinterpret_cast<double*>(take(b_vec));
    w.partial = reinterpret_cast<double*>(take(b_part));
    w.segD = reinterpret_cast<double*>(take(b_sd));
    w.hist = reinterpret_cast<double*>(take(b_hist));
    w.segI = reinterpret_cast<int*>(take(b_si));
    // every buffer is written before it is read (the first reductions set the CG scalars
    // and states of each problem), so nothing needs clearing
    const int st = pcg_run(c, b, x, rtol, maxit, w, false, t0);
    if (iters) *iters = c->stats.pcg_iters;
    if (relres) *relres = c->stats.pcg_relres;
    if (st == MSDD_ENOCONV) return code_for(c, MsddError{MSDD_ENOCONV, "PCG reached maxit"});
    return st;
  } catch (const MsddError& e) {
    return code_for(c, e);
  }
}

int msdd_solve(msdd_ctx* c, const double* b, double* x, double rtol, int32_t maxit,
               int32_t* iters, double* relres) {
  if (!c) return MSDD_EINVAL;
  if (!c->ready) return code_for(c, MsddError{MSDD_ESTATE, "msdd_solve before a successful setup"});
  try {
    const int st = solve_all(c, b, x, rtol, maxit);
    if (iters) *iters = c->stats.pcg_iters;
    if (relres) *relres = c->stats.pcg_relres;
    if (st == MSDD_ENOCONV) return code_for(c, MsddError{MSDD_ENOCONV, "PCG reached maxit"});
    return st;
  } catch (const MsddError& e) {
    return code_for(c, e);
  }
}

int msdd_solve_batch(msdd_ctx* c, const double* b, double* x, double rtol, int32_t maxit,
                     int32_t* iters, double* relres) {
  if (!c) return MSDD_EINVAL;
  if (!c->ready) return code_for(c, MsddError{MSDD_ESTATE, "msdd_solve_batch before a successful setup"});
  try {
    const int st = solve_all(c, b, x, rtol, maxit);
    for (int q = 0; q < c->nseg; ++q) {
      if (iters) iters[q] = c->last_iters[q];
      if (relres) relres[q] = c->last_relres[q];
    }
    if (st == MSDD_ENOCONV) return code_for(c, MsddError{MSDD_ENOCONV, "PCG reached maxit"});
    return st;
  } catch (const MsddError& e) {
    return code_for(c, e);
  }
}

int msdd_solve_history(const msdd_ctx* c, double* relres, int32_t cap, int32_t* count) {
  if (!c || !count || cap < 0) return MSDD_EINVAL;
  const int32_t nh = (int32_t)c->hist.size();
  *count = nh;
  if (relres)
    for (int32_t k = 0; k < std::min(nh, cap); ++k) relres[k] = c->hist[k];
  return MSDD_OK;
}

int msdd_stats(const msdd_ctx* c, msdd_stats_t* out) {
  if (!c || !out) return MSDD_EINVAL;
  *out = c->stats;
  return MSDD_OK;
}

int msdd_get_eig_iters(const msdd_ctx* c, int32_t* iters) {
  if (!c || !iters) return MSDD_EINVAL;
  if (!c->ready) return MSDD_ESTATE;
  msdd_ctx* cc = const_cast<msdd_ctx*>(c);
  try {
    HIPCHK(hipSetDevice(c->opt.device));
    const size_t P = c->eig_iters.size();
    HIPCHK(hipMemcpy(iters, c->eig_iters.data(), P * sizeof(int32_t),
                     is_device_ptr(iters) ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
  } catch (const MsddError& e) {
    return code_for(cc, e);
  }
  return MSDD_OK;
}

int msdd_autotune(msdd_ctx* c, int32_t what, int32_t reps) {
  if (!c) return MSDD_EINVAL;
  if (!c->ready) {
    set_err(c, "msdd_autotune needs a completed setup");
    return MSDD_ESTATE;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  try {
    HIPCHK(hipSetDevice(c->opt.device));
    REQUIRE(reps >= 1 && reps <= 100, "reps must lie in [1, 100]");
    REQUIRE((what & ~(MSDD_TUNE_EIG | MSDD_TUNE_SOLVE)) == 0 && what != 0, "bad tuning mask");
    hipStream_t s = c->stream;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // ms per launch of f: one untimed launch, then reps timed ones
    auto time_it = [&](const auto& f) -> float {
      f();
      HIPCHK(hipGetLastError());
      HIPCHK(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) f();
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      return ms / reps;
    };
    FineLevel& F = c->F;
    const int P = F.P;
    msdd_tuning_t& T = c->tune;
    // the eigensolver's launch shapes are those of the FP64 factor; a context set up with
    // the FP32 factor keeps the by-shape choice
    if ((what & MSDD_TUNE_EIG) && !F.eig32) {
      const int K = c->opt.block <= 16 ? 16 : (c->opt.block <= 32 ? 32 : 64);
      std::vector<int64_t> kvoff(P + 1, 0);
      for (int i = 0; i < P; ++i) kvoff[i + 1] = kvoff[i] + (int64_t)F.gs.h_n[i] * K;
      DVec<int64_t> dkvoff;
      dkvoff.upload(kvoff, s);
      DVec<double> W, Y, Z, GS, GB;
      W.alloc(kvoff.back());
      Y.alloc(kvoff.back());
      Z.alloc(kvoff.back());
      W.zero(s);
      Y.zero(s);
      Z.zero(s);
      for (float& v : T.eig_solve_ms) v = 0.f;
      int best = 0;
      // The eigensolver's launches run with every subdomain active at first and with few
      // at the end.  Each candidate is timed with all active (t_all) and with only the
      // subdomain that iterated longest (t_one, the latency of a lone subdomain); the
      // estimate per iteration weighs the two by the last setup's iteration counts,
      // sum over iterations k of t_one + (t_all - t_one) active(k) / P, over max_k.
      int i_long = 0;
      double it_sum = 0.0;
      for (int i = 0; i < (int)c->eig_iters.size() && i < P; ++i) {
        it_sum += c->eig_iters[i];
        if (c->eig_iters[i] > c->eig_iters[i_long]) i_long = i;
      }
      const double it_max = c->eig_iters.empty() ? 0.0 : (double)c->eig_iters[i_long];
      std::vector<int> st_one(P, ST_DONE);
      st_one[i_long] = ST_RUNNING;
      DVec<int> one;
      one.upload(st_one, s);
      for (int v = 1; v <= 9; ++v) {
        if ((v < 3 || (v > 3 && v < 8)) && F.bw_max >= 64) continue;  // rolling window: b < 64
        if (v >= 8 && !F.has_lb) continue;                              // blocked: b <= 64
        const float t_all = time_it([&] {
          eig_band_solve(c, s, dkvoff.p, K, W.p, Y.p, nullptr, v);
        });
        T.eig_solve_ms[v] = t_all;
        if (it_max > 0) {
          const float t_one = time_it([&] {
            eig_band_solve(c, s, dkvoff.p, K, W.p, Y.p, one.p, v);
          });
          T.eig_solve_ms[v] =
              (float)((it_max * t_one + (t_all - t_one) * it_sum / P) / it_max);
        }
        if (!best || T.eig_solve_ms[v] < T.eig_solve_ms[best]) best = v;
      }
      T.eig_solve = best;
      const int cand[5] = {1, 2, 4, 8, 16};
      GS.alloc((size_t)P * 16 * K * K);
      GB.alloc((size_t)P * 16 * K * K);
      int bs = 0;
      for (int q = 0; q < 5; ++q) {
        T.eig_splits_ms[q] = time_it([&] {
          launch_gram(s, P, F.gs.n.p, dkvoff.p, K, Y.p, W.p, Z.p, GS.p, GB.p, nullptr, cand[q]);
        });
        if (T.eig_splits_ms[q] < T.eig_splits_ms[bs]) bs = q;
      }
      T.eig_splits = cand[bs];
    }
    if (what & MSDD_TUNE_SOLVE) {
      const bool f32 = c->opt.precision == MSDD_MIXED;
      DVec<double> u;
      u.alloc(std::max<int64_t>(F.h_doff.back(), 1));
      u.zero(s);
      for (float& v : T.fine_solve_ms) v = 0.f;
      int best = 0;
      for (int v = 1; v <= 3; ++v) {
        if (v == 1 && F.bd_max >= 64) continue;  // rolling window needs a band below 64
        if (v == 3 && !F.twist_built) continue;  // two-sided factors built at the setup
        T.fine_solve_ms[v] = time_it([&] { fine_local_solve(c, s, u.p, v); });
        if (!best || T.fine_solve_ms[v] < T.fine_solve_ms[best]) best = v;
      }
      T.fine_solve = best;
      const int sgs[4] = {4, 8, 16, 32};
      int bs = 0;
      DVec<double> pv, qv;
      pv.alloc(c->n);
      qv.alloc(c->n);
      pv.zero(s);
      for (int q = 0; q < 4; ++q) {
        T.spmv_ms[q] = time_it([&] {
          launch_spmv_chunk(s, c->nch, sgs[q], c->ch_lo.p, c->ch_hi.p, c->rowptr.p, c->col.p,
                            c->val.p, pv.p, qv.p, c->partial.p);
        });
        if (T.spmv_ms[q] < T.spmv_ms[bs]) bs = q;
      }
      T.spmv_group = sgs[bs];
      c->spmv_sg = T.spmv_group;
      if (c->gexec) (void)hipGraphExecDestroy(c->gexec);  // captured with the old shapes
      c->gexec = nullptr;
    }
    HIPCHK(hipStreamSynchronize(s));
  } catch (const MsddError& e) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return code_for(c, e);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return MSDD_OK;
}

int msdd_get_tuning(const msdd_ctx* c, msdd_tuning_t* t) {
  if (!c || !t) return MSDD_EINVAL;
  *t = c->tune;
  return MSDD_OK;
}

int msdd_set_tuning(msdd_ctx* c, const msdd_tuning_t* t) {
  if (!c || !t) return MSDD_EINVAL;
  const bool ok = t->eig_solve >= 0 && t->eig_solve <= 9 && t->eig_splits >= 0 &&
                  t->eig_splits <= 16 && t->fine_solve >= 0 && t->fine_solve <= 3 &&
                  (t->spmv_group == 0 || t->spmv_group == 4 || t->spmv_group == 8 ||
                   t->spmv_group == 16 || t->spmv_group == 32);
  if (!ok) {
    set_err(c, "tuning value out of range");
    return MSDD_EINVAL;
  }
  c->tune.eig_solve = t->eig_solve;
  c->tune.eig_splits = t->eig_splits;
  c->tune.fine_solve = t->fine_solve;
  c->tune.spmv_group = t->spmv_group;
  if (c->ready && t->spmv_group > 0 && c->spmv_sg != t->spmv_group) {
    c->spmv_sg = t->spmv_group;
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  if (c->ready && c->gexec) {  // the fine-solve variant is part of the captured graph
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  return MSDD_OK;
}

int msdd_warm_start(msdd_ctx* c, msdd_net* net, int32_t n_sub, int32_t n_in, const float* x,
                    int64_t n_entries, const int32_t* sub_pos, int32_t n_pos, int32_t collect) {
  if (!c) return MSDD_EINVAL;
  try {
    HIPCHK(hipSetDevice(c->opt.device));
    auto& W = c->warm;
    if (n_sub == 0) {  // detach
      W.net = nullptr;
      W.P = 0;
      W.pos.clear();
      W.x.release();
      W.m_cap = 0;
      return MSDD_OK;
    }
    REQUIRE(n_sub > 0 && n_entries >= 0 && n_pos >= 1, "bad warm-start sizes");
    REQUIRE(collect >= 0 && collect <= 16, "collect must lie in [0, 16]");
    REQUIRE(net || collect > 0, "a warm start needs a network or collect > 0");
    if (net) {
      REQUIRE(msdd_net_internal::n_in(net) == n_in, "feature count differs from the network's n_in");
      REQUIRE(msdd_net_internal::n_pos(net) == n_pos, "frame size differs from the network's n_pos");
    }
    std::vector<int32_t> pos = to_host(sub_pos, (size_t)n_entries);
    for (int32_t v : pos) REQUIRE(v >= -1 && v < n_pos, "frame position out of range");
    if (net) {
      REQUIRE(n_in >= 1, "n_in must be positive");
      to_device(W.x, x, (size_t)n_sub * n_in, c->stream);
      HIPCHK(hipStreamSynchronize(c->stream));
    } else {
      W.x.release();
    }
    W.net = net;
    W.P = n_sub;
    W.n_in = n_in;
    W.n_pos = n_pos;
    W.m_cap = collect;
    W.n_entries = n_entries;
    W.pos = std::move(pos);
  } catch (const MsddError& e) {
    return code_for(c, e);
  }
  return MSDD_OK;
}

int msdd_warm_targets(const msdd_ctx* c, float* tgt, float* mask, int32_t* cnt) {
  if (!c) return MSDD_EINVAL;
  msdd_ctx* cc = const_cast<msdd_ctx*>(c);
  if (!c->ready || !c->warm.have_targets) {
    set_err(cc, "no training targets: run a setup with collect > 0 first");
    return MSDD_ESTATE;
  }
  try {
    HIPCHK(hipSetDevice(c->opt.device));
    REQUIRE(tgt && mask && cnt, "null output array");
    const auto& W = c->warm;
    auto cp = [&](void* dst, const void* src, size_t bytes) {
      HIPCHK(hipMemcpy(dst, src, bytes,
                       is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    };
    cp(tgt, W.tgt.p, W.tgt.n * sizeof(float));
    cp(mask, W.mask.p, W.mask.n * sizeof(float));
    cp(cnt, W.cnt.p, W.cnt.n * sizeof(int));
  } catch (const MsddError& e) {
    return code_for(cc, e);
  }
  return MSDD_OK;
}

int msdd_get_level_counts(const msdd_ctx* c, int32_t level, int32_t* m) {
  if (!c || !m || !c->ready) return MSDD_EINVAL;
  const int L = c->n_levels - 1;
  if (level == L) {
    for (size_t i = 0; i < c->F.m.size(); ++i) m[i] = c->F.m[i];
    return MSDD_OK;
  }
  for (const auto& CL : c->C)
    if (CL.level == level) {
      for (size_t i = 0; i < CL.m.size(); ++i) m[i] = CL.m[i];
      return MSDD_OK;
    }
  return MSDD_EINVAL;
}

int msdd_get_eigs(const msdd_ctx* c, int32_t level, int32_t i, int32_t n_extra, double* lam,
                  int32_t* count) {
  if (!c || !lam || !count || !c->ready || n_extra < 0) return MSDD_EINVAL;
  const int L = c->n_levels - 1;
  const std::vector<double>* src = nullptr;
  int m = 0;
  if (level == L) {
    if (i < 0 || i >= c->F.P) return MSDD_EINVAL;
    src = &c->F.lam[i];
    m = c->F.m[i];
  } else {
    for (const auto& CL : c->C)
      if (CL.level == level) {
        if (i < 0 || i >= CL.P) return MSDD_EINVAL;
        src = &CL.h_lam[i];
        m = CL.m[i];
      }
  }
  if (!src) return MSDD_EINVAL;
  const int cnt = std::min<int>((int)src->size(), m + n_extra);
  for (int a = 0; a < cnt; ++a) lam[a] = (*src)[a];
  *count = cnt;
  return MSDD_OK;
}

int msdd_get_basis(const msdd_ctx* c, int32_t level, int32_t i, double* basis, int32_t* rows,
                   int32_t* cols) {
  if (!c || !rows || !cols || !c->ready) return MSDD_EINVAL;
  const int L = c->n_levels - 1;
  try {
    if (level == L) {
      if (i < 0 || i >= c->F.P) return MSDD_EINVAL;
      *rows = c->F.gs.h_n[i];
      *cols = c->F.m[i];
      if (basis && (*rows) * (*cols) > 0)
        HIPCHK(hipMemcpy(basis, c->F.Phi.p + c->F.h_phi_off[i], sizeof(double) * (*rows) * (*cols),
                         hipMemcpyDeviceToHost));
      return MSDD_OK;
    }
    for (const auto& CL : c->C)
      if (CL.level == level) {
        if (i < 0 || i >= CL.P) return MSDD_EINVAL;
        *rows = CL.no[i];
        *cols = CL.m[i];
        if (basis && (*rows) * (*cols) > 0)
          HIPCHK(hipMemcpy(basis, CL.Y.p + CL.h_yoff[i], sizeof(double) * (*rows) * (*cols),
                           hipMemcpyDeviceToHost));
        return MSDD_OK;
      }
  } catch (const MsddError& e) {
    return e.code;
  }
  return MSDD_EINVAL;
}

int msdd_profile(msdd_ctx* c, int enable) {
  if (!c) return MSDD_EINVAL;
  try {
    if (enable == 1) c->prof.reset();
    c->prof.on = enable != 0;
    return MSDD_OK;
  } catch (const MsddError& e) {
    return code_for(c, e);
  }
}

int msdd_profile_query(msdd_ctx* c, int id, double* total_ms, int64_t* launches,
                       double* alg_bytes, double* alg_flops) {
  if (!c || id < 0 || id >= PR_COUNT) return MSDD_EINVAL;
  try {
    c->prof.resolve();
  } catch (const MsddError& e) {
    return code_for(c, e);
  }
  if (total_ms) *total_ms = c->prof.ms[id];
  if (launches) *launches = c->prof.cnt[id];
  if (alg_bytes) *alg_bytes = c->prof.bytes[id];
  if (alg_flops) *alg_flops = c->prof.flops[id];
  return MSDD_OK;
}

const char* msdd_profile_name(int id) { return (id >= 0 && id < PR_COUNT) ? kProfNames[id] : nullptr; }

const char* msdd_last_error(const msdd_ctx* c) { return c ? c->err.c_str() : "null context"; }

void msdd_destroy(msdd_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->opt.device);
  (void)hipDeviceSynchronize();
  delete c;
  DevicePool::get().safe_point();
}

}  // extern "C"
