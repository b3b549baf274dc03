// C ABI (include/bmg.h) and the host driver of BM-Global on one MI355X.
//
// The driver issues the kernels of kernels.hip on the problem's stream and
// keeps only q x q FP64 matrices and scalars on the host: the Gram matrices of
// the Rayleigh-Ritz step, of the orthonormalisation and of the exact SVD of the
// projected matrix, the Nystrom core, and the k x k preconditioner.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "batch.h"
#include "bmg.h"
#include "bmg_internal.h"

using namespace bmg;

// ============================================================================ errors
static thread_local std::string g_err;
static bmg_status fail(bmg_status s, const std::string &msg) {
  g_err = msg;
  return s;
}
extern "C" const char *bmg_last_error(void) { return g_err.c_str(); }
namespace bmg {
bmg_status set_error(bmg_status s, const std::string &msg) { return fail(s, msg); }
}  // namespace bmg

struct BmgError {
  bmg_status st;
  std::string msg;
};
#define HIPC(x)                                                                          \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      throw BmgError{BMG_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)};      \
  } while (0)
#define REQUIRE(cond, st, msg) \
  do {                         \
    if (!(cond)) throw BmgError{st, msg}; \
  } while (0)

// ============================================================================ host accounting
// Host time in the q x q linear algebra and in waits for the device, per solve
// (each solve runs on one host thread).
static thread_local double t_la_acc = 0.0, t_wait_acc = 0.0;
static thread_local int n_sync_acc = 0;
struct HostTimer {
  double &acc;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  explicit HostTimer(double &a) : acc(a) {}
  ~HostTimer() {
    acc += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};
// One helper thread for host work that can overlap the caller's: run() hands
// it a job, wait() returns once the job is done (started on first use).
struct HostHelper {
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  std::function<void()> job;
  bool has = false, done = true, quit = false;
  void loop() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv.wait(lk, [&] { return has || quit; });
      if (quit) return;
      std::function<void()> f = std::move(job);
      has = false;
      lk.unlock();
      f();
      lk.lock();
      done = true;
      cv.notify_all();
    }
  }
  void run(std::function<void()> f) {
    if (!th.joinable()) th = std::thread([this] { loop(); });
    std::lock_guard<std::mutex> g(mu);
    job = std::move(f);
    has = true;
    done = false;
    cv.notify_all();
  }
  void wait() {
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [&] { return done; });
  }
  ~HostHelper() {
    if (!th.joinable()) return;
    {
      std::lock_guard<std::mutex> g(mu);
      quit = true;
    }
    cv.notify_all();
    th.join();
  }
};
// waits for the helper's job when the scope ends (also on an exception)
struct HelperJoin {
  HostHelper &h;
  ~HelperJoin() { h.wait(); }
};

namespace lat {
inline void sym_eig(int n, const double *A, double *w, double *V) {
  HostTimer t(t_la_acc);
  la::sym_eig(n, A, w, V);
}
inline int chol_pivoted(int n, const double *G, double tol, int *perm, double *R) {
  HostTimer t(t_la_acc);
  return la::chol_pivoted(n, G, tol, perm, R);
}
inline bool chol(int n, const double *G, double *R) {
  HostTimer t(t_la_acc);
  return la::chol(n, G, R);
}
inline void tri_inv_upper(int n, const double *R, double *Rinv) {
  HostTimer t(t_la_acc);
  la::tri_inv_upper(n, R, Rinv);
}
inline bool spd_inv(int n, const double *A, double *Ainv) {
  HostTimer t(t_la_acc);
  return la::spd_inv(n, A, Ainv);
}
}  // namespace lat

// ============================================================================ constants
static constexpr double ORTH_TOL = 1e-6;   // numerical-rank cut of orth() on unit columns
static constexpr double SSI_EPS = 1e-12;   // Algorithm 2's cut of small s (relative)
static constexpr double PINV_REL = 1e-12;  // Nystrom pseudo-inverse cut (relative)
static constexpr double LMSVD_EIG_TOL = 1e-6;  // cut of small eigenvalues of P^T P (eq. PUi;
                                                // history columns have unit norm)
static constexpr int LMSVD_MAX_HIST = 4;       // largest history length p_t accepted
static constexpr uint64_t STREAM_SKETCH = 1, STREAM_SAFEGUARD = 0x100;

static inline int64_t rup(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// ============================================================================ workspace layout
struct Layout {
  int64_t m, n, nnz;
  int k_cap, ldk, qld, qmax;
  bool lowp;
  // persistent
  size_t csc_ptr, csc_idx, csc_a, perm, r_rows, r_cols, a32_rows, a32_cols;
  size_t pr_short, pr_long, pr_lp0, pr_prow, pr_pbeg, pr_pend, pr_pord;
  size_t pc_short, pc_long, pc_lp0, pc_prow, pc_pbeg, pc_pend, pc_pord;
  size_t wsum, wpart, partial, result, gram_part, small;
  size_t g_W, g_H, g_U, g_Y, d_W64, d_H64, d_R64;  // BF16 mode: shadows and FP64 refresh
  int64_t max_long, max_pieces, piece_bytes, wsum_cap, gram_cap;
  // scratch region (setup sort / solver blocks overlap)
  size_t scratch;
  size_t s_keys_out, s_vals_in, s_rid, s_temp, s_temp_bytes;
  size_t b_W, b_H, b_G, b_D, b_Wn, b_Hn, b_Ucur, b_Uprev, b_vec, b_B1, b_B2, b_B3, b_B4, b_Y, b_Y2;
  // variants reserved at creation: history blocks of Algorithm 2 (p_t <= hist_p)
  // and the state of the SpaRSA step rule
  int hist_p = 0;
  bool sparsa = false;
  size_t hist, hist_mb, hist_nb, sp, sp_bu, sp_bw, sp_bh, sp_br;
  // dense-row panel (reserved when the options ask for one): at most pn_max
  // rows of ldp columns, and the remainder of Omega without them in both
  // orientations (the rows side reuses the rows arrays with a plan of its own)
  double dense_rows = 0.0;
  int pn_max = 0;
  int64_t pn_ldi = 0, pn_part_cap = 0, pn_part2_cap = 0, pn_bsum_cap = 0;
  size_t pn_rows, pn_mask, pn_A64, pn_A32, pn_R, pn_part, pn_part2, pn_bsum, pn_xt;
  size_t prr_short, prr_long, prr_lp0, prr_prow, prr_pbeg, prr_pend, prr_pord;
  size_t cr_ptr, cr_idx, cr_a64, cr_a32, cr_r;
  size_t pcr_short, pcr_long, pcr_lp0, pcr_prow, pcr_pbeg, pcr_pend, pcr_pord;
  size_t s_keep, s_pos;
  size_t total;
};

static size_t sort_temp_bytes(int64_t nnz) {
  size_t bytes = 0, scan = 0;
  if (nnz <= 0) return 256;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t *)nullptr,
                                         (uint32_t *)nullptr, (const int32_t *)nullptr,
                                         (int32_t *)nullptr, (int)nnz, 0, 32,
                                         (hipStream_t)0) != hipSuccess)
    bytes = (size_t)nnz * 16;
  // the panel's compaction of the column-major orientation scans nnz flags
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, scan, (const int32_t *)nullptr, (int32_t *)nullptr,
                                       (int)nnz, (hipStream_t)0) != hipSuccess)
    scan = (size_t)nnz * 8;
  return std::max(bytes, scan) + 256;
}

static constexpr int PANEL_MAX_ROWS = 256;   // at most this many rows go to the dense panel

static Layout make_layout(int64_t m, int64_t n, int64_t nnz, int k_cap, bmg_precision prec,
                          int hist_p, bool sparsa, double dense_rows) {
  Layout L{};
  L.m = m; L.n = n; L.nnz = nnz; L.k_cap = k_cap;
  L.hist_p = hist_p;
  L.sparsa = sparsa;
  L.dense_rows = dense_rows;
  // leading dimensions in multiples of 16 elements: factor rows start on 128-byte lines
  L.ldk = (int)rup(std::max(k_cap, 1), 16);
  L.qmax = 2 * k_cap + 2;
  L.qld = (int)rup(L.qmax, 16);
  L.lowp = prec != BMG_FP64;
  L.max_long = nnz / LONG_ROW + 1;
  // every piece but the last of its row holds at least PIECE_MIN entries
  L.max_pieces = nnz / PIECE_MIN + L.max_long + 1;
  // one scalar slot per wave of a row-kernel grid (two runs padded to 8 blocks)
  L.wsum_cap = std::max(m, n) + L.max_pieces + 80;
  L.gram_cap = std::max<int64_t>(64LL * L.qmax * L.qmax, 2048LL * 4096);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += rup((int64_t)bytes + 1, 256); return o; };
  L.csc_ptr = take(8 * (n + 1));
  L.csc_idx = take(4 * nnz);
  L.csc_a = take(8 * nnz);
  L.perm = take(4 * nnz);
  L.r_rows = take(8 * nnz);
  L.r_cols = take(8 * nnz);
  L.a32_rows = take(L.lowp ? 4 * nnz : 0);
  L.a32_cols = take(L.lowp ? 4 * nnz : 0);
  L.pr_short = take(4 * m);
  L.pr_long = take(4 * L.max_long);
  L.pr_lp0 = take(4 * (L.max_long + 1));
  L.pr_prow = take(4 * L.max_pieces);
  L.pr_pbeg = take(8 * L.max_pieces);
  L.pr_pend = take(8 * L.max_pieces);
  L.pr_pord = take(4 * L.max_pieces);
  L.pc_short = take(4 * n);
  L.pc_long = take(4 * L.max_long);
  L.pc_lp0 = take(4 * (L.max_long + 1));
  L.pc_prow = take(4 * L.max_pieces);
  L.pc_pbeg = take(8 * L.max_pieces);
  L.pc_pend = take(8 * L.max_pieces);
  L.pc_pord = take(4 * L.max_pieces);
  L.wsum = take(16 * L.wsum_cap);
  L.wpart = take(16 * 256);
  {
    // widest partial row of any pass slice (padded to whole lane-group chunks)
    const int es = prec == BMG_FP64 ? 8 : 4;
    const int wmax = std::min(L.qmax, prec == BMG_FP64 ? max_width<double>() : max_width<float>());
    L.piece_bytes = (int64_t)wmax * es <= 1024 ? 1024 : 2048;
  }
  L.partial = take((size_t)L.max_pieces * L.piece_bytes);
  L.result = take(8 * 64);
  L.gram_part = take(8 * L.gram_cap);
  L.small = take(8 * 9 * (size_t)L.qld * L.qld);
  {
    const bool bf = prec == BMG_BF16;
    const int64_t mi0 = std::min(m, n), ni0 = std::max(m, n);
    L.g_W = take(bf ? 2 * mi0 * L.ldk : 0);
    L.g_H = take(bf ? 2 * ni0 * L.ldk : 0);
    L.g_U = take(bf ? 2 * mi0 * L.qld : 0);
    L.g_Y = take(bf ? 2 * ni0 * L.qld : 0);
    L.d_W64 = take(bf ? 8 * mi0 * L.ldk : 0);
    L.d_H64 = take(bf ? 8 * ni0 * L.ldk : 0);
    L.d_R64 = take(bf ? 8 * nnz : 0);
  }
  {
    // element size of the solver's blocks in this precision
    const int64_t es = prec == BMG_FP64 ? 8 : 4;
    const int64_t mi0 = std::min(m, n), ni0 = std::max(m, n);
    // history: (2p - 1) short-side and 3p long-side blocks of qld columns
    L.hist_mb = (size_t)rup(es * mi0 * L.qld, 256);
    L.hist_nb = (size_t)rup(es * ni0 * L.qld, 256);
    L.hist = take(hist_p > 0 ? (size_t)(2 * hist_p - 1) * L.hist_mb + (size_t)(3 * hist_p) * L.hist_nb : 0);
    // SpaRSA: the kept warm start, the previous PG point W, H, its residual and
    // the sampled values of X~
    L.sp_bu = (size_t)rup(es * mi0 * L.qld, 256);
    L.sp_bw = (size_t)rup(es * mi0 * L.ldk, 256);
    L.sp_bh = (size_t)rup(es * ni0 * L.ldk, 256);
    L.sp_br = (size_t)rup(es * std::max<int64_t>(nnz, 1), 256);
    L.sp = take(sparsa ? L.sp_bu + L.sp_bw + L.sp_bh + 2 * L.sp_br : 0);
  }
  {
    // dense-row panel: rows with at least dense_rows * n entries, so at most
    // nnz / (dense_rows n) of them (and at most PANEL_MAX_ROWS, the densest)
    const int64_t mi0 = std::min(m, n), ni0 = std::max(m, n);
    int64_t pmax = 0;
    if (dense_rows > 0.0 && dense_rows <= 1.0 && ni0 > 0)
      pmax = std::min<int64_t>({PANEL_MAX_ROWS, mi0, (int64_t)((double)nnz / (dense_rows * (double)ni0))});
    L.pn_max = (int)std::max<int64_t>(pmax, 0);
    const bool pn = L.pn_max > 0;
    L.pn_ldi = rup(std::max(L.pn_max, 1), 16);
    const int64_t cells = pn ? L.pn_ldi * std::max<int64_t>(ni0, 1) : 0;
    L.pn_part_cap = pn ? (int64_t)PANEL_KSPLIT * L.pn_ldi * L.qld : 0;
    L.pn_part2_cap = pn ? (int64_t)PANEL_KGROUPS * L.pn_ldi * L.qld : 0;
    L.pn_bsum_cap = pn ? (ni0 + 15) / 16 : 0;
    L.pn_rows = take(pn ? 4 * L.pn_ldi : 0);
    L.pn_mask = take(pn ? mi0 : 0);
    L.pn_A64 = take(8 * cells);
    L.pn_A32 = take(L.lowp ? 4 * cells : 0);
    L.pn_R = take(8 * cells);
    L.pn_part = take(8 * L.pn_part_cap);
    L.pn_part2 = take(8 * L.pn_part2_cap);
    L.pn_bsum = take(16 * L.pn_bsum_cap);
    L.pn_xt = take(pn ? 8 * L.pn_ldi * L.qld : 0);
    L.prr_short = take(pn ? 4 * mi0 : 0);
    L.prr_long = take(pn ? 4 * L.max_long : 0);
    L.prr_lp0 = take(pn ? 4 * (L.max_long + 1) : 0);
    L.prr_prow = take(pn ? 4 * L.max_pieces : 0);
    L.prr_pbeg = take(pn ? 8 * L.max_pieces : 0);
    L.prr_pend = take(pn ? 8 * L.max_pieces : 0);
    L.prr_pord = take(pn ? 4 * L.max_pieces : 0);
    L.cr_ptr = take(pn ? 8 * (ni0 + 1) : 0);
    L.cr_idx = take(pn ? 4 * nnz : 0);
    L.cr_a64 = take(pn ? 8 * nnz : 0);
    L.cr_a32 = take(pn && L.lowp ? 4 * nnz : 0);
    L.cr_r = take(pn ? 8 * nnz : 0);
    L.pcr_short = take(pn ? 4 * ni0 : 0);
    L.pcr_long = take(pn ? 4 * L.max_long : 0);
    L.pcr_lp0 = take(pn ? 4 * (L.max_long + 1) : 0);
    L.pcr_prow = take(pn ? 4 * L.max_pieces : 0);
    L.pcr_pbeg = take(pn ? 8 * L.max_pieces : 0);
    L.pcr_pend = take(pn ? 8 * L.max_pieces : 0);
    L.pcr_pord = take(pn ? 4 * L.max_pieces : 0);
  }
  L.scratch = off;
  // setup view of the scratch region
  size_t so = off;
  auto stake = [&](size_t bytes) { size_t o = so; so += rup((int64_t)bytes + 1, 256); return o; };
  L.s_keys_out = stake(4 * nnz);
  L.s_vals_in = stake(4 * nnz);
  L.s_rid = stake(4 * nnz);
  L.s_temp_bytes = sort_temp_bytes(nnz);
  L.s_temp = stake(L.s_temp_bytes);
  L.s_keep = stake(4 * nnz);
  L.s_pos = stake(4 * nnz);
  // solver view of the scratch region (element size 8 regardless of precision);
  // the solver runs on the orientation with mi = min(m, n) rows
  size_t bo = off;
  auto btake = [&](size_t elems) { size_t o = bo; bo += rup((int64_t)(8 * elems) + 1, 256); return o; };
  const int64_t mi = std::min(m, n), ni = std::max(m, n);
  L.b_W = btake(mi * L.ldk);
  L.b_H = btake(ni * L.ldk);
  L.b_G = btake(ni * L.ldk);
  L.b_D = btake(ni * L.ldk);
  L.b_Wn = btake(mi * L.ldk);
  L.b_Hn = btake(ni * L.ldk);
  L.b_Ucur = btake(mi * L.ldk);
  L.b_Uprev = btake(mi * L.ldk);
  L.b_vec = btake(8 * rup(ni, 64));
  L.b_B1 = btake(mi * L.qld);
  L.b_B2 = btake(mi * L.qld);
  L.b_B3 = btake(mi * L.qld);
  L.b_B4 = btake(mi * L.qld);
  L.b_Y = btake(ni * L.qld);
  L.b_Y2 = btake(ni * L.qld);
  L.total = std::max(so, bo);
  return L;
}

// ============================================================================ problem
struct Side {  // one orientation of Omega
  Plan pl;
  const double *a64 = nullptr;
  float *a32 = nullptr;
  void *r = nullptr;  // stored residual in this orientation's order (T)
};

// ============================================================================ pass batcher
// A pass waits in the queue until every attached problem has a pass queued or
// BATCH_WINDOW_S has passed since it was queued; then the first queued pass
// of its kind (precision, mode, width class) launches up to BATCH_MAX passes
// of that kind together, in queue order.
static constexpr double BATCH_WINDOW_S = 100e-6;

struct bmg::PassBatcher {
  struct Item {
    int key = 0, prec = 0, mode = 0;
    PassArg<double, double> a64;
    PassArg<float, float> a32;
    PassArg<float, bf16_t> a16;
    hipEvent_t ready = nullptr, done = nullptr;   // owned by the problem
    bool taken = false, finished = false;
    hipError_t err = hipSuccess;
  };
  std::mutex mu;
  std::condition_variable cv;
  hipStream_t bs = nullptr;
  int attached = 0;
  long launches = 0, passes = 0;
  std::deque<Item *> q;

  hipError_t launch(std::vector<Item *> &b) {
    hipError_t e = hipSuccess;
    for (Item *x : b)
      if (e == hipSuccess) e = hipStreamWaitEvent(bs, x->ready, 0);
    if (e != hipSuccess) return e;
    const int n = (int)b.size(), mode = b[0]->mode;
    if (b[0]->prec == 0) {
      PassArg<double, double> d[BATCH_MAX];
      for (int i = 0; i < n; ++i) d[i] = b[i]->a64;
      e = launch_batch<double, double>(d, n, mode, bs);
    } else if (b[0]->prec == 1) {
      PassArg<float, float> d[BATCH_MAX];
      for (int i = 0; i < n; ++i) d[i] = b[i]->a32;
      e = launch_batch<float, float>(d, n, mode, bs);
    } else {
      PassArg<float, bf16_t> d[BATCH_MAX];
      for (int i = 0; i < n; ++i) d[i] = b[i]->a16;
      e = launch_batch<float, bf16_t>(d, n, mode, bs);
    }
    for (Item *x : b)
      if (e == hipSuccess) e = hipEventRecord(x->done, bs);
    return e;
  }

  // Queues the pass (its inputs are ready once `s` reaches this point) and
  // returns when it is launched, with `s` made to wait for its completion.
  hipError_t submit(Item &it, hipStream_t s) {
    hipError_t e = hipEventRecord(it.ready, s);
    if (e != hipSuccess) return e;
    std::unique_lock<std::mutex> lk(mu);
    it.taken = it.finished = false;
    it.err = hipSuccess;
    q.push_back(&it);
    const auto until = std::chrono::steady_clock::now() +
                       std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                           std::chrono::duration<double>(BATCH_WINDOW_S));
    cv.notify_all();
    while (!it.taken) {
      Item *lead = nullptr;
      for (Item *x : q)
        if (x->key == it.key) { lead = x; break; }
      if (lead != &it) {
        cv.wait(lk);
        continue;
      }
      cv.wait_until(lk, until, [&] { return it.taken || (int)q.size() >= attached; });
      if (it.taken) break;
      std::vector<Item *> b;
      for (auto i = q.begin(); i != q.end() && (int)b.size() < BATCH_MAX;) {
        if ((*i)->key == it.key) {
          (*i)->taken = true;
          b.push_back(*i);
          i = q.erase(i);
        } else {
          ++i;
        }
      }
      lk.unlock();
      const hipError_t le = launch(b);
      lk.lock();
      launches += 1;
      passes += (long)b.size();
      for (Item *x : b) {
        x->err = le;
        x->finished = true;
      }
      cv.notify_all();
    }
    cv.wait(lk, [&] { return it.finished; });
    e = it.err;
    lk.unlock();
    if (e == hipSuccess) e = hipStreamWaitEvent(s, it.done, 0);
    return e;
  }
};

struct bmg_problem {
  Layout L;
  bmg_precision prec;
  hipStream_t s;
  char *ws;
  int64_t m_user, n_user, nnz;
  bool transposed;  // internal problem is the transpose (user m > n)
  Side urow, ucol;  // user CSR orientation and the built column orientation
  int32_t *perm;    // column-order position -> CSR position
  // dense-row panel of the internal rows (P = 0: none) and Omega without its
  // rows: prow shares the internal rows' arrays (own plan), pcol has its own
  // column-major arrays
  int panel_P = 0, panel_ldi = 0;
  int32_t *panel_rows = nullptr;
  double *panel_A64 = nullptr;
  float *panel_A32 = nullptr;
  void *panel_R = nullptr;
  Side prow, pcol;
  double *result, *gram_part, *small;
  double *wsum, *wpart;
  // pinned host staging of the solver's small transfers (q x q Gram matrices
  // down, small coefficient matrices up): a fetch area of hpin_fetch doubles,
  // then a ring of hpin_ring doubles for uploads, free again after every
  // synchronisation of the stream.  Null when pinning failed (pageable copies).
  double *hpin = nullptr, *hpin_dev = nullptr;  // host address, device address
  size_t hpin_fetch = 0, hpin_ring = 0, hpin_off = 0;
  void *partial;
  // serving: sparse passes go through a shared batcher when set
  PassBatcher *batcher = nullptr;
  PassBatcher::Item bitem;
  // statistics of the sparse passes since the last reset
  double bytes = 0.0;
  int passes = 0;
  int bf16_passes = 0;     // passes that gathered BF16 copies of their operand
  bool pass_bf16 = false;  // the pass being issued gathers BF16
  // kernel timing with HIP events (opt->timing)
  struct Pend {
    hipEvent_t a, b;
    int cls;
    double bytes;
  };
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<Pend> pend;
  hipEvent_t last_a = nullptr, last_b = nullptr;
  int last_cls = 0;
  double kms[3] = {0, 0, 0}, kbytes[3] = {0, 0, 0};
  int klaunch[3] = {0, 0, 0};
  hipEvent_t get_event() {
    if (ev_pool.empty()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      return e;
    }
    hipEvent_t e = ev_pool.back();
    ev_pool.pop_back();
    return e;
  }
  void resolve_timing() {  // call after the stream has been synchronised
    for (const Pend &q : pend) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
        kms[q.cls] += ms;
        kbytes[q.cls] += q.bytes;
        klaunch[q.cls] += 1;
      }
      ev_pool.push_back(q.a);
      ev_pool.push_back(q.b);
    }
    pend.clear();
  }
  void reset_stats() {
    bytes = 0.0;
    passes = 0;
    bf16_passes = 0;
    for (int i = 0; i < 3; ++i) kms[i] = kbytes[i] = 0.0, klaunch[i] = 0;
  }
  ~bmg_problem() {
    if (hpin) (void)hipHostFree(hpin);
    for (const Pend &q : pend) { (void)hipEventDestroy(q.a); (void)hipEventDestroy(q.b); }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (bitem.ready) (void)hipEventDestroy(bitem.ready);
    if (bitem.done) (void)hipEventDestroy(bitem.done);
  }

  template <typename T> T *at(size_t off) { return reinterpret_cast<T *>(ws + off); }
  Side &rows() { return transposed ? ucol : urow; }  // internal rows (short side)
  Side &cols() { return transposed ? urow : ucol; }
  int64_t mi() { return transposed ? n_user : m_user; }
  int64_t ni() { return transposed ? m_user : n_user; }
  PassScratch scratch() {
    PassScratch sc;
    sc.wsum = wsum;
    sc.wpart = wpart;
    sc.partial = partial;
    sc.partial_bytes = (int64_t)L.max_pieces * L.piece_bytes;
    sc.result = result;
    return sc;
  }
};

// Where the plan's device arrays live in the workspace.
struct PlanSlots {
  size_t shorts, longs, lp0, prow, pbeg, pend, pord;
};

// skip (optional, host, nrows): rows left out of the plan (the panel's rows)
static void build_plan(bmg_problem *P, int64_t nrows, int64_t ncols, const int64_t *d_ptr,
                       const int32_t *d_idx, const PlanSlots &o, Plan &pl,
                       const std::vector<uint8_t> *skip = nullptr) {
  std::vector<int64_t> ptr(nrows + 1);
  HIPC(hipMemcpyAsync(ptr.data(), d_ptr, 8 * (nrows + 1), hipMemcpyDeviceToHost, P->s));
  HIPC(hipStreamSynchronize(P->s));
  auto len = [&](int64_t r) { return ptr[r + 1] - ptr[r]; };
  std::vector<int32_t> shorts, longs;
  shorts.reserve(nrows);
  int64_t nnz_plan = 0;
  for (int64_t i = 0; i < nrows; ++i) {
    if (skip && (*skip)[i]) continue;
    nnz_plan += len(i);
    if (len(i) <= LONG_ROW) shorts.push_back((int32_t)i);
    else longs.push_back((int32_t)i);
  }
  std::stable_sort(shorts.begin(), shorts.end(),
                   [&](int32_t a, int32_t b) { return len(a) > len(b); });
  const int64_t n_long = (int64_t)longs.size();
  REQUIRE(n_long <= P->L.max_long, BMG_EINVAL, "plan larger than its bound");
  if (!shorts.empty())
    HIPC(hipMemcpyAsync(P->at<int32_t>(o.shorts), shorts.data(), 4 * shorts.size(),
                        hipMemcpyHostToDevice, P->s));
  if (n_long > 0)
    HIPC(hipMemcpyAsync(P->at<int32_t>(o.longs), longs.data(), 4 * longs.size(),
                        hipMemcpyHostToDevice, P->s));
  // --- column ranges and where each long row crosses them (computed on the GPU
  // into the setup scratch: n_long (nr + 1) < nnz int32 fit its 4 nnz bytes)
  const int nr = (int)std::max<int64_t>(
      1, std::min<int64_t>(MAX_RANGES, (ncols + RANGE_COLS - 1) / RANGE_COLS));
  const int64_t wc = std::max<int64_t>(1, (ncols + nr - 1) / nr);
  std::vector<int32_t> bnd((size_t)n_long * (nr + 1));
  if (n_long > 0) {
    int32_t *d_bnd = P->at<int32_t>(P->L.s_keys_out);
    HIPC(launch_range_bounds(d_ptr, d_idx, P->at<int32_t>(o.longs), n_long, nr, wc, d_bnd, P->s));
    HIPC(hipMemcpyAsync(bnd.data(), d_bnd, 4 * bnd.size(), hipMemcpyDeviceToHost, P->s));
    HIPC(hipStreamSynchronize(P->s));
  }
  // --- pieces, row by row: at most LONG_ROW entries, cut at a range end once
  // they hold PIECE_MIN entries; key = column range of the first entry
  std::vector<int32_t> lp0, prow, pkey;
  std::vector<int64_t> pbeg, pend;
  for (int64_t i = 0; i < n_long; ++i) {
    const int32_t r = longs[i];
    const int32_t *B = &bnd[(size_t)i * (nr + 1)];
    const int64_t L = len(r), base = ptr[r];
    lp0.push_back((int32_t)prow.size());
    auto emit = [&](int64_t b, int64_t e, int key) {
      prow.push_back(r);
      pbeg.push_back(base + b);
      pend.push_back(base + e);
      pkey.push_back(key);
    };
    int64_t cur = 0;
    int sk = 0;
    for (int kr = 0; kr < nr; ++kr) {
      const int64_t ek = kr + 1 < nr ? (int64_t)B[kr + 1] : L;
      while (ek - cur > LONG_ROW) {
        emit(cur, cur + LONG_ROW, sk);
        cur += LONG_ROW;
        sk = kr;
      }
      if (ek - cur >= PIECE_MIN) {
        emit(cur, ek, sk);
        cur = ek;
        sk = kr + 1;
      }
    }
    if (cur < L) emit(cur, L, std::min(sk, nr - 1));
  }
  lp0.push_back((int32_t)prow.size());
  const int64_t n_pieces = (int64_t)prow.size();
  REQUIRE(n_pieces <= P->L.max_pieces, BMG_EINVAL, "plan larger than its bound");
  // launch order: by key (counting sort; stable in piece order)
  std::vector<int32_t> pord(n_pieces);
  {
    std::vector<int64_t> start(nr + 1, 0);
    for (int32_t k : pkey) ++start[k + 1];
    for (int kr = 0; kr < nr; ++kr) start[kr + 1] += start[kr];
    for (int64_t pc = 0; pc < n_pieces; ++pc) pord[start[pkey[pc]]++] = (int32_t)pc;
  }
  HIPC(hipMemcpyAsync(P->at<int32_t>(o.lp0), lp0.data(), 4 * lp0.size(), hipMemcpyHostToDevice,
                      P->s));
  if (n_pieces > 0) {
    HIPC(hipMemcpyAsync(P->at<int32_t>(o.prow), prow.data(), 4 * n_pieces, hipMemcpyHostToDevice,
                        P->s));
    HIPC(hipMemcpyAsync(P->at<int64_t>(o.pbeg), pbeg.data(), 8 * n_pieces, hipMemcpyHostToDevice,
                        P->s));
    HIPC(hipMemcpyAsync(P->at<int64_t>(o.pend), pend.data(), 8 * n_pieces, hipMemcpyHostToDevice,
                        P->s));
    HIPC(hipMemcpyAsync(P->at<int32_t>(o.pord), pord.data(), 4 * n_pieces, hipMemcpyHostToDevice,
                        P->s));
  }
  HIPC(hipStreamSynchronize(P->s));  // host vectors go out of scope
  pl.nrows = nrows;
  pl.ncols = ncols;
  pl.nnz = nnz_plan;
  pl.ptr = d_ptr;
  pl.idx = d_idx;
  pl.short_rows = P->at<int32_t>(o.shorts);
  pl.n_short = (int64_t)shorts.size();
  pl.long_rows = P->at<int32_t>(o.longs);
  pl.long_p0 = P->at<int32_t>(o.lp0);
  pl.n_long = n_long;
  pl.piece_row = P->at<int32_t>(o.prow);
  pl.piece_beg = P->at<int64_t>(o.pbeg);
  pl.piece_end = P->at<int64_t>(o.pend);
  pl.piece_ord = P->at<int32_t>(o.pord);
  pl.n_pieces = n_pieces;
}

// Dense-row panel of the internal rows: the rows with at least dense_rows * n
// entries (the densest pn_max of them), their values as a dense panel (NaN
// where nothing is observed), and the plans of Omega without them: the
// internal rows' arrays with those rows skipped, and a compacted copy of the
// column-major orientation without their entries.
static void build_panel(bmg_problem *P) {
  const Layout &L = P->L;
  Side &Rw = P->rows(), &Cl = P->cols();
  const int64_t mi = P->mi(), ni = P->ni(), nnz = P->nnz;
  std::vector<int64_t> ptr(mi + 1);
  HIPC(hipMemcpyAsync(ptr.data(), Rw.pl.ptr, 8 * (mi + 1), hipMemcpyDeviceToHost, P->s));
  HIPC(hipStreamSynchronize(P->s));
  const double thr = L.dense_rows * (double)ni;
  std::vector<std::pair<int64_t, int32_t>> cand;
  for (int64_t i = 0; i < mi; ++i) {
    const int64_t len = ptr[i + 1] - ptr[i];
    if (len > 0 && (double)len >= thr) cand.push_back({-len, (int32_t)i});
  }
  std::sort(cand.begin(), cand.end());
  if ((int64_t)cand.size() > L.pn_max) cand.resize(L.pn_max);
  std::vector<int32_t> rows;
  for (auto &c : cand) rows.push_back(c.second);
  std::sort(rows.begin(), rows.end());
  if (rows.empty()) return;
  const int Pn = (int)rows.size();
  const int ldi = (int)rup(Pn, 16);
  while ((int)rows.size() < ldi) rows.push_back(rows[0]);   // padding slots (unobserved)
  P->panel_ldi = ldi;
  P->panel_rows = P->at<int32_t>(L.pn_rows);
  P->panel_A64 = P->at<double>(L.pn_A64);
  P->panel_A32 = L.lowp ? P->at<float>(L.pn_A32) : nullptr;
  P->panel_R = P->at<void>(L.pn_R);
  std::vector<uint8_t> skip(mi, 0);
  for (int32_t r : rows) skip[r] = 1;
  uint8_t *mask = P->at<uint8_t>(L.pn_mask);
  HIPC(hipMemcpyAsync(P->panel_rows, rows.data(), 4 * ldi, hipMemcpyHostToDevice, P->s));
  HIPC(hipMemcpyAsync(mask, skip.data(), mi, hipMemcpyHostToDevice, P->s));
  HIPC(launch_panel_fill(Pn, ni, ldi, P->panel_rows, Rw.pl.ptr, Rw.pl.idx, Rw.a64, P->panel_A64,
                         P->panel_A32, P->s));
  // rows of Omega without the panel's: the same arrays, a plan of their own
  build_plan(P, mi, ni, Rw.pl.ptr, Rw.pl.idx,
             {L.prr_short, L.prr_long, L.prr_lp0, L.prr_prow, L.prr_pbeg, L.prr_pend, L.prr_pord},
             P->prow.pl, &skip);
  P->prow.a64 = Rw.a64;
  P->prow.a32 = Rw.a32;
  P->prow.r = Rw.r;
  // column-major orientation without the panel's entries (order kept)
  int32_t *keep = P->at<int32_t>(L.s_keep), *pos = P->at<int32_t>(L.s_pos);
  int64_t *cptr = P->at<int64_t>(L.cr_ptr);
  int32_t *cidx = P->at<int32_t>(L.cr_idx);
  double *ca = P->at<double>(L.cr_a64);
  HIPC(launch_panel_keep(nnz, Cl.pl.idx, mask, keep, P->s));
  size_t tb = L.s_temp_bytes;
  HIPC(hipcub::DeviceScan::ExclusiveSum(P->at<void>(L.s_temp), tb, keep, pos, (int)nnz, P->s));
  HIPC(launch_panel_compact(ni, nnz, Cl.pl.ptr, keep, pos, Cl.pl.idx, Cl.a64, cidx, ca, cptr, P->s));
  HIPC(hipStreamSynchronize(P->s));
  build_plan(P, ni, mi, cptr, cidx,
             {L.pcr_short, L.pcr_long, L.pcr_lp0, L.pcr_prow, L.pcr_pbeg, L.pcr_pend, L.pcr_pord},
             P->pcol.pl);
  P->pcol.a64 = ca;
  P->pcol.r = P->at<void>(L.cr_r);
  if (L.lowp) {
    P->pcol.a32 = P->at<float>(L.cr_a32);
    HIPC((launch_convert<double, float>(P->pcol.pl.nnz, ca, P->pcol.a32, P->s)));
  }
  P->panel_P = Pn;
}

// ============================================================================ typed solver
// Everything below runs on the internal orientation: m <= n, rows() = Omega,
// cols() = Omega^T.  T is the storage/multiply type of the sparse passes.
template <typename T, typename TG = T>
struct Engine {
  static constexpr bool kShadow = !std::is_same<T, TG>::value;
  // BF16 mode: the subspace products of a refresh step gather the FP32 masters
  bool exact_gather = false;
  bmg_problem *P;
  hipStream_t s;
  int ldk, qld;
  int64_t m, n;
  Side *R, *C;
  // dense-row panel: its rows leave the sparse passes (Rr, Cr: Omega without
  // them) and go through the panel kernels; never with BF16 gathers or shared
  // launches, and switched off by the solver variants that read the stored
  // residual entry by entry (polyMF-SS, SpaRSA)
  bool panel_on = false;
  Side *Rr = nullptr, *Cr = nullptr;
  PanelArg<T> pa;

  explicit Engine(bmg_problem *p) : P(p), s(p->s), ldk(p->L.ldk), qld(p->L.qld) {
    m = P->mi();
    n = P->ni();
    R = &P->rows();
    C = &P->cols();
    if (P->panel_P > 0 && !kShadow && !P->batcher) {
      panel_on = true;
      Rr = &P->prow;
      Cr = &P->pcol;
      pa.P = P->panel_P;
      pa.n = n;
      pa.ldi = P->panel_ldi;
      pa.rows = P->panel_rows;
      if constexpr (sizeof(T) == 8) pa.A = (const T *)P->panel_A64;
      else pa.A = (const T *)P->panel_A32;
      pa.R = (T *)P->panel_R;
    }
  }
  // panel residual of X_P Y^T (sums into result[4..5])
  void panel_resid(const T *Xm, int ldx, const T *Yn, int ldy, int k, bool use_a, bool store) {
    HIPC(launch_panel_resid<T>(pa, Xm, ldx, Yn, ldy, k, use_a, store, P->template at<double>(P->L.pn_bsum),
                               P->L.pn_bsum_cap, P->wpart, P->result + 4, s));
  }
  void panel_rows(bool values, const T *Y, int ldy, int q, double coef, const T *X, int ldx, int kx,
                  const T *M, int ldm, double lam, const T *Xl, T *Out, int ldo) {
    HIPC(launch_panel_rows<T>(pa, values, Y, ldy, q, coef, X, ldx, kx, M, ldm, lam, Xl, ldk, Out, ldo,
                              P->template at<double>(P->L.pn_part), P->L.pn_part_cap,
                              P->template at<double>(P->L.pn_part2), P->L.pn_part2_cap, s));
  }
  const T *avals(Side *sd) {
    if constexpr (sizeof(T) == 8) return (const T *)sd->a64;
    else return (const T *)sd->a32;
  }
  // Runs f(gathered operand): the BF16 shadow of src, or src itself in the FP64 /
  // FP32 modes and whenever exact_gather is set.
  template <class F>
  void with_gather(int slot, const T *src, int64_t rows, int cols, int ld, F &&f) {
    if constexpr (kShadow) {
      if (!exact_gather) {
        P->pass_bf16 = true;
        f(gath(slot, src, rows, cols, ld));
        return;
      }
    }
    f(src);
  }
  // The operand a sparse pass gathers, in the gather type: src itself, or its
  // BF16 shadow (converted just before the pass).  Slots: 0 m-side factor,
  // 1 n-side factor, 2 m-side block, 3 n-side block.
  const TG *gath(int slot, const T *src, int64_t rows, int cols, int ld) {
    if constexpr (!kShadow) {
      return src;
    } else {
      const size_t off = slot == 0 ? P->L.g_W : slot == 1 ? P->L.g_H : slot == 2 ? P->L.g_U : P->L.g_Y;
      TG *dst = P->at<TG>(off);
      if (cols > 0 && rows > 0) HIPC((launch_convert_cols<T, TG>(rows, cols, src, ld, dst, ld, s)));
      return dst;
    }
  }
  T *blk(size_t off) { return P->at<T>(off); }

  // scratch for one sparse pass of kernel class cls (events attached when timing)
  PassScratch sx(int cls) {
    PassScratch sc = P->scratch();
    if (P->timing) {
      sc.ev0 = P->last_a = P->get_event();
      sc.ev1 = P->last_b = P->get_event();
      P->last_cls = cls;
      if (panel_on) {
        // the events bracket the sparse kernel and the panel kernels of the pass
        HIPC(hipEventRecord(sc.ev0, s));
        sc.ev0 = sc.ev1 = nullptr;
      }
    }
    return sc;
  }
  // algorithmic bytes of the pass over the whole of Omega (the panel's own
  // traffic is not counted); pl is the full plan of the orientation
  void count(const Plan &pl, double per_nnz, double fixed) {
    const double b = per_nnz * (double)pl.nnz + fixed + 8.0 * (double)(pl.nrows + 1);
    P->bytes += b;
    P->passes += 1;
    P->bf16_passes += P->pass_bf16 ? 1 : 0;
    P->pass_bf16 = false;
    if (panel_on && P->timing && P->last_b) HIPC(hipEventRecord(P->last_b, s));
    if (P->timing && P->last_a && P->last_b) {
      P->pend.push_back({P->last_a, P->last_b, P->last_cls, b});
      P->last_a = P->last_b = nullptr;
    }
  }
  void fetch(double *h, const double *d, size_t cnt) {
    const bool pin = P->hpin && cnt <= P->hpin_fetch;
    HIPC(hipMemcpyAsync(pin ? P->hpin : h, d, 8 * cnt, hipMemcpyDeviceToHost, s));
    {
      HostTimer t(t_wait_acc);
      HIPC(hipStreamSynchronize(s));
    }
    if (pin) memcpy(h, P->hpin, 8 * cnt);
    P->hpin_off = 0;  // every upload queued so far has completed
    n_sync_acc += 1;
    if (!P->pend.empty()) P->resolve_timing();
  }
  // ---------------------------------------------------------------- dense helpers
  std::vector<double> gram(int64_t N, int a, const T *X, int ldx, int b, const T *Y, int ldy) {
    std::vector<double> h((size_t)a * b, 0.0);
    if (a == 0 || b == 0) return h;
    if (P->hpin_dev && (size_t)a * b <= P->hpin_fetch) {
      // the final reduction writes straight into the pinned fetch area
      HIPC(launch_gram<T>(N, a, X, ldx, b, Y, ldy, P->gram_part, P->L.gram_cap, P->hpin_dev, s));
      {
        HostTimer t(t_wait_acc);
        HIPC(hipStreamSynchronize(s));
      }
      memcpy(h.data(), P->hpin, 8 * h.size());
      P->hpin_off = 0;
      n_sync_acc += 1;
      if (!P->pend.empty()) P->resolve_timing();
      return h;
    }
    HIPC(launch_gram<T>(N, a, X, ldx, b, Y, ldy, P->gram_part, P->L.gram_cap, P->small, s));
    fetch(h.data(), P->small, (size_t)a * b);
    return h;
  }
  // X^T Y (a x b) into device staging slot `slot` as T, without a host round trip
  T *gram_dev(int64_t N, int a, const T *X, int ldx, int b, const T *Y, int ldy, int slot) {
    double *d = P->small + (size_t)(slot + 1) * P->L.qld * P->L.qld;
    REQUIRE((size_t)a * b <= (size_t)P->L.qld * P->L.qld, BMG_EINVAL, "small matrix too large");
    if (a == 0 || b == 0) return (T *)d;
    if constexpr (sizeof(T) == 8) {
      HIPC(launch_gram<T>(N, a, X, ldx, b, Y, ldy, P->gram_part, P->L.gram_cap, d, s));
    } else {
      HIPC(launch_gram<T>(N, a, X, ldx, b, Y, ldy, P->gram_part, P->L.gram_cap, P->small, s));
      HIPC((launch_convert<double, T>((int64_t)a * b, P->small, (T *)d, s)));
    }
    return (T *)d;
  }
  // host source of an upload of `bytes`: a slot of the pinned ring holding a
  // copy of src (queued copies from it run asynchronously), or src itself
  const void *stage_up(const void *src, size_t bytes) {
    const size_t cnt = (bytes + 255) / 256 * 32;  // doubles, 256-byte granules
    if (!P->hpin || cnt > P->hpin_ring) return src;
    if (P->hpin_off + cnt > P->hpin_ring) {  // ring full: wait for its copies
      HostTimer t(t_wait_acc);
      HIPC(hipStreamSynchronize(s));
      P->hpin_off = 0;
    }
    double *dst = P->hpin + P->hpin_fetch + P->hpin_off;
    P->hpin_off += cnt;
    memcpy(dst, src, bytes);
    return dst;
  }
  // upload a small FP64 matrix into the device staging area (slot 0..7)
  double *put(const std::vector<double> &h, int slot) {
    double *d = P->small + (size_t)(slot + 1) * P->L.qld * P->L.qld;
    REQUIRE(h.size() <= (size_t)P->L.qld * P->L.qld, BMG_EINVAL, "small matrix too large");
    if (!h.empty())
      HIPC(hipMemcpyAsync(d, stage_up(h.data(), 8 * h.size()), 8 * h.size(), hipMemcpyHostToDevice, s));
    return d;
  }
  // same, converted to T (for the low-rank epilogue of the sparse products)
  T *put_t(const std::vector<double> &h, int slot) {
    if constexpr (sizeof(T) == 8) {
      return (T *)put(h, slot);
    } else {
      std::vector<float> f(h.begin(), h.end());
      T *d = (T *)(P->small + (size_t)(slot + 1) * P->L.qld * P->L.qld);
      if (!f.empty())
        HIPC(hipMemcpyAsync(d, stage_up(f.data(), 4 * f.size()), 4 * f.size(), hipMemcpyHostToDevice, s));
      return d;
    }
  }
  void gemm(int64_t N, int a, const T *X, int ldx, int b, const std::vector<double> &M, T *Cm,
            int ldc, double beta, int slot = 7) {
    if (b == 0 || N == 0) return;
    const double *dM = put(M, slot);
    HIPC(launch_gemm_ts<T>(N, a, X, ldx, b, dM, b, Cm, ldc, beta, s));
  }
  // ---------------------------------------------------------------- pass dispatch
  // mode 0 fused residual + product, 1 sampled residual, 2 sparse x dense
  // (arguments as in launch_grad / launch_sddmm / launch_spmm).  Through the
  // problem's batcher when it has one and the width fits one lane-group slice.
  template <typename TY>
  void pass(int mode, const Plan &pl, const T *a, const T *X, int ldx, const TY *Y, int ldy,
            int width, double lam, double coef, T *out, int ldo, int kx, const T *M, int ldm,
            PassScratch sc) {
    if (P->batcher && width <= max_width<T>()) {
      PassArg<T, TY> d;
      d.pl = pl;
      d.a = a; d.X = X; d.Y = Y; d.M = M; d.out = out;
      d.partial = (T *)sc.partial; d.wsum = sc.wsum; d.result = sc.result;
      d.partial_bytes = sc.partial_bytes;
      d.lam = lam; d.coef = coef;
      d.ldx = ldx; d.ldy = ldy; d.width = width; d.ldo = ldo; d.kx = kx; d.ldm = ldm;
      PassBatcher::Item &it = P->bitem;
      if (!it.ready) HIPC(hipEventCreateWithFlags(&it.ready, hipEventDisableTiming));
      if (!it.done) HIPC(hipEventCreateWithFlags(&it.done, hipEventDisableTiming));
      it.mode = mode;
      if constexpr (std::is_same<T, double>::value) { it.prec = 0; it.a64 = d; }
      else if constexpr (std::is_same<TY, float>::value) { it.prec = 1; it.a32 = d; }
      else { it.prec = 2; it.a16 = d; }
      it.key = (it.prec * 4 + mode) * 1024 + width_class<TY>(width);
      HIPC(P->batcher->submit(it, s));
      return;
    }
    if (mode == 0)
      HIPC((launch_grad<T, TY>(pl, a, X, ldx, Y, ldy, width, lam, out, ldo, sc, nullptr, s)));
    else if (mode == 1)
      HIPC((launch_sddmm<T, TY>(pl, a, X, ldx, Y, ldy, width, out, sc, s)));
    else
      HIPC((launch_spmm<T, TY>(pl, a, Y, ldy, width, coef, X, ldx, kx, M, ldm, out, ldo, sc, s)));
  }

  // ---------------------------------------------------------------- sparse passes
  // BM gradient on the rows side: G = R H + lam W (+ f = 1/2 sum r^2)
  double grad_rows(const T *W, const T *H, int k, double lam, T *G) {
    if (panel_on) {
      // rows of Omega without the panel's, then the panel's rows: R_P stored,
      // G_P = R_P H + lam W_P
      pass<T>(0, Rr->pl, avals(R), W, ldk, H, ldk, k, lam, 0.0, G, ldk, 0, nullptr, 0, sx(0));
      panel_resid(W, ldk, H, ldk, k, true, true);
      panel_rows(false, H, ldk, k, 1.0, nullptr, 0, 0, nullptr, 0, lam, W, G, ldk);
      count(R->pl, 4.0 + sizeof(T), (double)n * k * sizeof(TG) + 2.0 * m * k * sizeof(T));
      double h[6];
      fetch(h, P->result, 6);
      return 0.5 * (h[0] + h[4]);
    }
    with_gather(1, H, n, k, ldk, [&](auto Yg) {
      using TY = std::remove_const_t<std::remove_pointer_t<decltype(Yg)>>;
      pass<TY>(0, R->pl, avals(R), W, ldk, Yg, ldk, k, lam, 0.0, G, ldk, 0, nullptr, 0, sx(0));
    });
    count(R->pl, 4.0 + sizeof(T), (double)n * k * sizeof(TG) + 2.0 * m * k * sizeof(T));
    double h[1];
    fetch(h, P->result, 1);
    return 0.5 * h[0];
  }
  double grad_cols(const T *W, const T *H, int k, double lam, T *G) {
    if (panel_on) {
      // columns without the panel's entries (G = R^T W + lam H), then G += R_P^T W_P
      pass<T>(0, Cr->pl, avals(Cr), H, ldk, W, ldk, k, lam, 0.0, G, ldk, 0, nullptr, 0, sx(0));
      panel_resid(W, ldk, H, ldk, k, true, true);
      HIPC(launch_panel_cols<T>(pa, false, W, ldk, k, 1.0, G, ldk, P->template at<T>(P->L.pn_xt), s));
      count(C->pl, 4.0 + sizeof(T), (double)m * k * sizeof(TG) + 2.0 * n * k * sizeof(T));
      double h[6];
      fetch(h, P->result, 6);
      return 0.5 * (h[0] + h[4]);
    }
    with_gather(0, W, m, k, ldk, [&](auto Yg) {
      using TY = std::remove_const_t<std::remove_pointer_t<decltype(Yg)>>;
      pass<TY>(0, C->pl, avals(C), H, ldk, Yg, ldk, k, lam, 0.0, G, ldk, 0, nullptr, 0, sx(0));
    });
    count(C->pl, 4.0 + sizeof(T), (double)m * k * sizeof(TG) + 2.0 * n * k * sizeof(T));
    double h[1];
    fetch(h, P->result, 1);
    return 0.5 * h[0];
  }
  // sum over Omega of (x_row . y_col)^2 on the given side
  double curvature(Side *sd, const T *X, const T *Y, int k, int64_t nx, int64_t ny) {
    if (panel_on) {
      const bool rows_side = sd == R;
      pass<T>(1, rows_side ? Rr->pl : Cr->pl, (const T *)nullptr, X, ldk, Y, ldk, k, 0.0, 0.0, (T *)nullptr,
              0, 0, nullptr, 0, sx(1));
      // the panel's entries: (x_i . y_j)^2 with x the m-side operand
      if (rows_side) panel_resid(X, ldk, Y, ldk, k, false, false);
      else panel_resid(Y, ldk, X, ldk, k, false, false);
      count(sd->pl, 4.0, (double)nx * k * sizeof(T) + (double)ny * k * sizeof(TG));
      double h[6];
      fetch(h, P->result, 6);
      return h[0] + h[4];
    }
    with_gather(sd == R ? 1 : 0, Y, ny, k, ldk, [&](auto Yg) {
      using TY = std::remove_const_t<std::remove_pointer_t<decltype(Yg)>>;
      pass<TY>(1, sd->pl, (const T *)nullptr, X, ldk, Yg, ldk, k, 0.0, 0.0, (T *)nullptr, 0, 0,
               nullptr, 0, sx(1));
    });
    count(sd->pl, 4.0, (double)nx * k * sizeof(T) + (double)ny * k * sizeof(TG));
    double h[2];
    fetch(h, P->result, 2);
    return h[0];
  }
  // stored residual on one side; returns {sum r^2, sum r (r + a)}
  void sddmm_store(Side *sd, const T *X, const T *Y, int k, int64_t nx, int64_t ny, double out[2]) {
    if (panel_on) {
      if (sd == R) {
        // rows without the panel's into the rows' residual array, the panel's into R_P
        pass<T>(1, Rr->pl, avals(R), X, ldk, Y, ldk, k, 0.0, 0.0, (T *)R->r, 0, 0, nullptr, 0, sx(1));
        panel_resid(X, ldk, Y, ldk, k, true, true);
        count(R->pl, 4.0 + 2.0 * sizeof(T), (double)nx * k * sizeof(T) + (double)ny * k * sizeof(TG));
        double h[6];
        fetch(h, P->result, 6);
        out[0] = h[0] + h[4];
        out[1] = h[1] + h[5];
      } else {
        // the columns' copy holds the entries outside the panel only (the
        // panel's residual is shared by both orientations): sums of those
        pass<T>(1, Cr->pl, avals(Cr), X, ldk, Y, ldk, k, 0.0, 0.0, (T *)Cr->r, 0, 0, nullptr, 0, sx(1));
        count(C->pl, 4.0 + 2.0 * sizeof(T), (double)nx * k * sizeof(T) + (double)ny * k * sizeof(TG));
        fetch(out, P->result, 2);
      }
      return;
    }
    with_gather(sd == R ? 1 : 0, Y, ny, k, ldk, [&](auto Yg) {
      using TY = std::remove_const_t<std::remove_pointer_t<decltype(Yg)>>;
      pass<TY>(1, sd->pl, avals(sd), X, ldk, Yg, ldk, k, 0.0, 0.0, (T *)sd->r, 0, 0, nullptr, 0,
               sx(1));
    });
    count(sd->pl, 4.0 + 2.0 * sizeof(T), (double)nx * k * sizeof(T) + (double)ny * k * sizeof(TG));
    fetch(out, P->result, 2);
  }
  // 1/2 sum over Omega of (w_i . h_j - v_p)^2 for values v in CSR order
  double loss_vs(const T *v, const T *W, const T *H, int k) {
    if (R->pl.nnz == 0) return 0.0;
    REQUIRE(!panel_on, BMG_EINVAL, "entrywise sampled values are not available with a dense-row panel");
    with_gather(1, H, n, k, ldk, [&](auto Yg) {
      using TY = std::remove_const_t<std::remove_pointer_t<decltype(Yg)>>;
      pass<TY>(1, R->pl, v, W, ldk, Yg, ldk, k, 0.0, 0.0, (T *)nullptr, 0, 0, nullptr, 0, sx(1));
    });
    count(R->pl, 4.0 + sizeof(T), (double)m * k * sizeof(T) + (double)n * k * sizeof(TG));
    double h[2];
    fetch(h, P->result, 2);
    return 0.5 * h[0];
  }
  double loss(const T *W, const T *H, int k) {
    if (R->pl.nnz == 0) return 0.0;
    if (panel_on) {
      pass<T>(1, Rr->pl, avals(R), W, ldk, H, ldk, k, 0.0, 0.0, (T *)nullptr, 0, 0, nullptr, 0, sx(1));
      panel_resid(W, ldk, H, ldk, k, true, false);
      count(R->pl, 4.0 + sizeof(T), (double)m * k * sizeof(T) + (double)n * k * sizeof(TG));
      double h[6];
      fetch(h, P->result, 6);
      return 0.5 * (h[0] + h[4]);
    }
    with_gather(1, H, n, k, ldk, [&](auto Yg) {
      using TY = std::remove_const_t<std::remove_pointer_t<decltype(Yg)>>;
      pass<TY>(1, R->pl, avals(R), W, ldk, Yg, ldk, k, 0.0, 0.0, (T *)nullptr, 0, 0, nullptr, 0,
               sx(1));
    });
    count(R->pl, 4.0 + sizeof(T), (double)m * k * sizeof(T) + (double)n * k * sizeof(TG));
    double h[2];
    fetch(h, P->result, 2);
    return 0.5 * h[0];
  }

  // ---------------------------------------------------------------- Z operator
  // Z = X~ - alpha * S with X~ = W H^T (k columns, may be 0) and S the stored
  // values of each side (residual, or -A for the initialisation).
  struct ZOp {
    const T *W, *H;
    int k;
    double alpha;
    const T *s_rows, *s_cols;
    bool values = false;  // S is the observed values (else the stored residual)
  };
  // Y (n x q) = Z^T U = H (W^T U) - alpha S^T U
  void z_t(const ZOp &z, const T *U, int q, T *Y) {
    if (q == 0) return;
    T *dM = nullptr;
    if (z.k > 0) dM = gram_dev(m, z.k, z.W, ldk, q, U, qld, 0);
    if (panel_on) {
      const T *sc = z.values ? avals(Cr) : (const T *)Cr->r;
      pass<T>(2, Cr->pl, sc, z.H, ldk, U, qld, q, 0.0, -z.alpha, Y, qld, z.k, dM, q, sx(2));
      HIPC(launch_panel_cols<T>(pa, z.values, U, qld, q, -z.alpha, Y, qld, P->template at<T>(P->L.pn_xt), s));
      count(C->pl, 4.0 + sizeof(T), (double)m * q * sizeof(TG) + (double)n * q * sizeof(T));
      return;
    }
    with_gather(2, U, m, q, qld, [&](auto Ug) {
      using TY = std::remove_const_t<std::remove_pointer_t<decltype(Ug)>>;
      pass<TY>(2, C->pl, z.s_cols, z.H, ldk, Ug, qld, q, 0.0, -z.alpha, Y, qld, z.k, dM, q, sx(2));
    });
    count(C->pl, 4.0 + sizeof(T), (double)m * q * sizeof(TG) + (double)n * q * sizeof(T));
  }
  // V (m x q) = Z Y = W (H^T Y) - alpha S Y
  // (Y and V at leading dimension ld, qld when not given)
  void z_n(const ZOp &z, const T *Y, int q, T *V, int ld = 0) {
    if (q == 0) return;
    const int l = ld > 0 ? ld : qld;
    T *dM = nullptr;
    if (z.k > 0) dM = gram_dev(n, z.k, z.H, ldk, q, Y, l, 1);
    if (panel_on) {
      pass<T>(2, Rr->pl, z.s_rows, z.W, ldk, Y, l, q, 0.0, -z.alpha, V, l, z.k, dM, q, sx(2));
      panel_rows(z.values, Y, l, q, -z.alpha, z.W, ldk, z.k, dM, q, 0.0, nullptr, V, l);
      count(R->pl, 4.0 + sizeof(T), (double)n * q * sizeof(TG) + (double)m * q * sizeof(T));
      return;
    }
    with_gather(3, Y, n, q, l, [&](auto Yg) {
      using TY = std::remove_const_t<std::remove_pointer_t<decltype(Yg)>>;
      pass<TY>(2, R->pl, z.s_rows, z.W, ldk, Yg, l, q, 0.0, -z.alpha, V, l, z.k, dM, q, sx(2));
    });
    count(R->pl, 4.0 + sizeof(T), (double)n * q * sizeof(TG) + (double)m * q * sizeof(T));
  }

  // ---------------------------------------------------------------- orth
  // Orthonormal basis of ran(M) (N x c, ld qld) into U (ld qld), using tmp.
  // Unit-normalised columns, pivoted Cholesky of their Gram matrix with the
  // numerical-rank cut |R_jj| > ORTH_TOL, then one Cholesky re-orthogonalisation.
  int orth(int64_t N, const T *M, int c, T *U, T *tmp) {
    if (c == 0) return 0;
    std::vector<double> G = gram(N, c, M, qld, c, M, qld);
    std::vector<int> nz;
    std::vector<double> dn;
    for (int i = 0; i < c; ++i)
      if (G[(size_t)i * c + i] > 0.0) {
        nz.push_back(i);
        dn.push_back(sqrt(G[(size_t)i * c + i]));
      }
    const int c2 = (int)nz.size();
    if (c2 == 0) return 0;
    std::vector<double> Gn((size_t)c2 * c2), Rp((size_t)c2 * c2);
    for (int i = 0; i < c2; ++i)
      for (int j = 0; j < c2; ++j)
        Gn[(size_t)i * c2 + j] = G[(size_t)nz[i] * c + nz[j]] / (dn[i] * dn[j]);
    std::vector<int> perm(c2);
    const int r = lat::chol_pivoted(c2, Gn.data(), ORTH_TOL * ORTH_TOL, perm.data(), Rp.data());
    if (r == 0) return 0;
    std::vector<double> R11((size_t)r * r), Ri((size_t)r * r);
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < r; ++j) R11[(size_t)i * r + j] = (j >= i) ? Rp[(size_t)i * c2 + j] : 0.0;
    lat::tri_inv_upper(r, R11.data(), Ri.data());
    std::vector<double> Cm((size_t)c * r, 0.0);  // Q1 = M Cm
    for (int jj = 0; jj < r; ++jj) {
      const int col = nz[perm[jj]];
      const double sc = 1.0 / dn[perm[jj]];
      for (int l = 0; l < r; ++l) Cm[(size_t)col * r + l] = sc * Ri[(size_t)jj * r + l];
    }
    gemm(N, c, M, qld, r, Cm, tmp, qld, 0.0);
    // re-orthogonalise
    std::vector<double> G2 = gram(N, r, tmp, qld, r, tmp, qld), R2((size_t)r * r), R2i((size_t)r * r);
    if (!lat::chol(r, G2.data(), R2.data())) {
      // loss of orthogonality beyond repair by one pass: fall back to a second pivoted pass
      std::vector<int> p2(r);
      std::vector<double> Rq((size_t)r * r);
      const int r2 = lat::chol_pivoted(r, G2.data(), 1e-14, p2.data(), Rq.data());
      REQUIRE(r2 > 0, BMG_ENONFINITE, "orthonormalisation broke down");
      std::vector<double> Q11((size_t)r2 * r2), Qi((size_t)r2 * r2), C2((size_t)r * r2, 0.0);
      for (int i = 0; i < r2; ++i)
        for (int j = 0; j < r2; ++j) Q11[(size_t)i * r2 + j] = (j >= i) ? Rq[(size_t)i * r + j] : 0.0;
      lat::tri_inv_upper(r2, Q11.data(), Qi.data());
      for (int jj = 0; jj < r2; ++jj)
        for (int l = 0; l < r2; ++l) C2[(size_t)p2[jj] * r2 + l] = Qi[(size_t)jj * r2 + l];
      gemm(N, r, tmp, qld, r2, C2, U, qld, 0.0);
      return r2;
    }
    lat::tri_inv_upper(r, R2.data(), R2i.data());
    gemm(N, r, tmp, qld, r, R2i, U, qld, 0.0);
    return r;
  }
};

// ============================================================================ C ABI: setup
extern "C" void bmg_options_default(bmg_options *o) {
  memset(o, 0, sizeof(*o));
  o->lambda = 1.0;
  o->alpha = 1.99;
  o->tol = 1e-6;
  o->ssi_tol_floor = 1e-12;
  o->psi0 = 0.1;
  o->bm_epochs = 3;
  o->max_iter = 500;
  o->ssi_max_iter = 50;
  o->k_init = 8;
  o->refresh_every = 5;
  o->verbose = 0;
  o->lmsvd_p = 0;
  o->seed = 0;
  o->step_rule = BMG_STEP_FIXED;
  o->bm_solver = BMG_BM_POLYMF;
  o->alpha_min = 1.99;
  o->alpha_max = 1e3;
  o->sparsa_beta = 0.5;
  o->sparsa_delta = 0.999;
  o->dense_rows = 0.0;
}

// history length, step rule and dense-row threshold the workspace reserves
// for (opt may be null)
static bool reserve_of(const bmg_options *opt, int *hist_p, bool *sparsa, double *dense_rows) {
  *hist_p = opt ? opt->lmsvd_p : 0;
  *sparsa = opt && opt->step_rule == BMG_STEP_SPARSA;
  *dense_rows = opt ? opt->dense_rows : 0.0;
  return *hist_p >= 0 && *hist_p <= LMSVD_MAX_HIST && *dense_rows >= 0.0 && *dense_rows <= 1.0;
}

extern "C" bmg_status bmg_workspace_size(int64_t m, int64_t n, int64_t nnz, int k_cap,
                                         bmg_precision prec, const bmg_options *opt, size_t *bytes) {
  if (!bytes || m < 0 || n < 0 || nnz < 0 || k_cap < 1 || nnz > (int64_t)INT32_MAX ||
      m > (int64_t)INT32_MAX || n > (int64_t)INT32_MAX)
    return fail(BMG_EINVAL, "bmg_workspace_size: bad shape");
  if (prec != BMG_FP64 && prec != BMG_FP32 && prec != BMG_BF16) return fail(BMG_EINVAL, "unknown precision");
  const int64_t mi = std::min(m, n);
  (void)mi;
  if (k_cap > (prec == BMG_FP64 ? max_width<double>() : max_width<float>()))
    return fail(BMG_EINVAL, "k_cap above the widest sparse-pass slice");
  int hp = 0;
  bool sp = false;
  double dr = 0.0;
  if (!reserve_of(opt, &hp, &sp, &dr)) return fail(BMG_EINVAL, "lmsvd_p outside [0, 4] or dense_rows outside [0, 1]");
  Layout L = make_layout(m, n, nnz, k_cap, prec, hp, sp, dr);
  *bytes = L.total;
  return BMG_OK;
}

extern "C" bmg_status bmg_problem_create(const bmg_csr *csr, int k_cap, bmg_precision prec,
                                         const bmg_options *opt, void *ws, size_t ws_bytes,
                                         void *stream, bmg_problem **out) {
  if (!csr || !out || !ws) return fail(BMG_EINVAL, "bmg_problem_create: null argument");
  *out = nullptr;
  size_t need = 0;
  bmg_status st = bmg_workspace_size(csr->m, csr->n, csr->nnz, k_cap, prec, opt, &need);
  if (st != BMG_OK) return st;
  if (ws_bytes < need) return fail(BMG_ENOMEM, "workspace smaller than bmg_workspace_size");
  if (csr->m == 0 || csr->n == 0) return fail(BMG_EINVAL, "empty matrix shape");
  if (csr->nnz > 0 && (!csr->row_ptr || !csr->col || !csr->val))
    return fail(BMG_EINVAL, "null CSR array");
  bmg_problem *P = new bmg_problem();
  try {
    int hp = 0;
    bool sp = false;
    double dr = 0.0;
    reserve_of(opt, &hp, &sp, &dr);
    P->L = make_layout(csr->m, csr->n, csr->nnz, k_cap, prec, hp, sp, dr);
    P->prec = prec;
    P->s = (hipStream_t)stream;
    P->ws = (char *)ws;
    P->m_user = csr->m;
    P->n_user = csr->n;
    P->nnz = csr->nnz;
    P->transposed = csr->m > csr->n;
    const Layout &L = P->L;
    const int64_t m = csr->m, n = csr->n, nnz = csr->nnz;
    P->perm = P->at<int32_t>(L.perm);
    P->result = P->at<double>(L.result);
    P->gram_part = P->at<double>(L.gram_part);
    P->small = P->at<double>(L.small);
    P->wsum = P->at<double>(L.wsum);
    P->wpart = P->at<double>(L.wpart);
    P->partial = P->at<void>(L.partial);
    {
      const size_t q2 = (size_t)L.qld * L.qld;
      if (hipHostMalloc((void **)&P->hpin, 8 * 3 * q2, hipHostMallocDefault) == hipSuccess) {
        if (hipHostGetDevicePointer((void **)&P->hpin_dev, P->hpin, 0) != hipSuccess) {
          P->hpin_dev = nullptr;
          (void)hipGetLastError();
        }
        P->hpin_fetch = q2;
        P->hpin_ring = 2 * q2;
      } else {
        P->hpin = nullptr;
        (void)hipGetLastError();
      }
    }
    // --- validate the CSR (row ids first; they also feed the transpose)
    int32_t *rid = P->at<int32_t>(L.s_rid);
    int64_t nnz_dev = 0;
    HIPC(hipMemcpyAsync(&nnz_dev, csr->row_ptr + m, 8, hipMemcpyDeviceToHost, P->s));
    int64_t first = 0;
    HIPC(hipMemcpyAsync(&first, csr->row_ptr, 8, hipMemcpyDeviceToHost, P->s));
    HIPC(hipStreamSynchronize(P->s));
    REQUIRE(nnz_dev == nnz && first == 0, BMG_EINVAL, "row_ptr[0] != 0 or row_ptr[m] != nnz");
    int *flags = (int *)P->result;
    HIPC(hipMemsetAsync(flags, 0, sizeof(int), P->s));
    if (nnz > 0) {
      HIPC(launch_row_ids(m, csr->row_ptr, rid, P->s));
      HIPC(launch_check_csr(m, n, csr->row_ptr, csr->col, csr->val, rid, flags, P->s));
    }
    int hflags = 0;
    HIPC(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, P->s));
    HIPC(hipStreamSynchronize(P->s));
    REQUIRE(!(hflags & 4), BMG_ENONFINITE, "non-finite observed value");
    REQUIRE(!(hflags & 8), BMG_EINVAL, "row_ptr decreases");
    REQUIRE(!(hflags & 2), BMG_EINVAL, "column index out of range");
    REQUIRE(!(hflags & 1), BMG_EINVAL, "columns not strictly increasing within a row");
    // --- column-major copy: stable radix sort of the column indices (CSR order
    // is row-major, so each column's entries come out in increasing row order)
    int64_t *cptr = P->at<int64_t>(L.csc_ptr);
    int32_t *cidx = P->at<int32_t>(L.csc_idx);
    double *ca = P->at<double>(L.csc_a);
    if (nnz > 0) {
      uint32_t *keys_out = P->at<uint32_t>(L.s_keys_out);
      int32_t *vals_in = P->at<int32_t>(L.s_vals_in);
      HIPC(launch_iota(nnz, vals_in, P->s));
      int bits = 1;
      while ((int64_t(1) << bits) < n) ++bits;
      size_t tb = L.s_temp_bytes;
      HIPC(hipcub::DeviceRadixSort::SortPairs(P->at<void>(L.s_temp), tb, (const uint32_t *)csr->col,
                                              keys_out, vals_in, P->perm, (int)nnz, 0, bits, P->s));
      HIPC(launch_col_ptr(nnz, n, (const int32_t *)keys_out, cptr, P->s));
      HIPC(launch_gather_csc(nnz, P->perm, rid, csr->val, cidx, ca, P->s));
    } else {
      HIPC(launch_fill<int64_t>(cptr, n + 1, 1, 1, 0.0, P->s));
    }
    HIPC(hipStreamSynchronize(P->s));
    // --- plans
    build_plan(P, m, n, csr->row_ptr, csr->col,
               {L.pr_short, L.pr_long, L.pr_lp0, L.pr_prow, L.pr_pbeg, L.pr_pend, L.pr_pord},
               P->urow.pl);
    build_plan(P, n, m, cptr, cidx,
               {L.pc_short, L.pc_long, L.pc_lp0, L.pc_prow, L.pc_pbeg, L.pc_pend, L.pc_pord},
               P->ucol.pl);
    P->urow.a64 = csr->val;
    P->ucol.a64 = ca;
    P->urow.r = P->at<void>(L.r_rows);
    P->ucol.r = P->at<void>(L.r_cols);
    if (prec != BMG_FP64) {
      P->urow.a32 = P->at<float>(L.a32_rows);
      P->ucol.a32 = P->at<float>(L.a32_cols);
      HIPC((launch_convert<double, float>(nnz, csr->val, P->urow.a32, P->s)));
      HIPC((launch_convert<double, float>(nnz, ca, P->ucol.a32, P->s)));
    }
    if (L.pn_max > 0 && nnz > 0) build_panel(P);
    HIPC(hipStreamSynchronize(P->s));
  } catch (const BmgError &e) {
    delete P;
    return fail(e.st, e.msg);
  }
  *out = P;
  return BMG_OK;
}

extern "C" void bmg_problem_destroy(bmg_problem *p) { delete p; }

// ============================================================================ C ABI: primitives (FP64)
static bmg_status check_factors(bmg_problem *P, const void *W, const void *H, int k, int ld) {
  if (!P) return fail(BMG_EINVAL, "null problem");
  if (k < 0 || k > P->L.k_cap || ld < k || ld % 8 != 0) return fail(BMG_EINVAL, "bad k / ld");
  if (k > 0 && (!W || !H)) return fail(BMG_EINVAL, "null factor");
  if ((((uintptr_t)W) & 15) || (((uintptr_t)H) & 15)) return fail(BMG_EINVAL, "factors not 16-byte aligned");
  return BMG_OK;
}

extern "C" bmg_status bmg_sddmm(bmg_problem *P, const double *W, const double *H, int k, int ld,
                                double *R, double *half_sq) {
  bmg_status st = check_factors(P, W, H, k, ld);
  if (st != BMG_OK) return st;
  try {
    double h[2] = {0, 0};
    if (P->nnz > 0) {
      HIPC((launch_sddmm<double, double>(P->urow.pl, P->urow.a64, W, ld, H, ld, k, R, P->scratch(), P->s)));
      HIPC(hipMemcpyAsync(h, P->result, 16, hipMemcpyDeviceToHost, P->s));
    }
    HIPC(hipStreamSynchronize(P->s));
    if (half_sq) *half_sq = 0.5 * h[0];
  } catch (const BmgError &e) {
    return fail(e.st, e.msg);
  }
  return BMG_OK;
}

extern "C" bmg_status bmg_spmm(bmg_problem *P, const double *S, const double *B, int q, int ldb,
                               double *C, int ldc, int transpose) {
  if (!P || q < 0 || ldb < q || ldc < q || ldb % 2 || ldc % 2) return fail(BMG_EINVAL, "bmg_spmm: bad argument");
  try {
    if (q == 0) return BMG_OK;
    if (!transpose) {
      if (P->nnz == 0) HIPC(launch_fill<double>(C, P->m_user, q, ldc, 0.0, P->s));
      else HIPC((launch_spmm<double, double>(P->urow.pl, S, B, ldb, q, 1.0, nullptr, 0, 0, nullptr, 0, C, ldc,
                                    P->scratch(), P->s)));
    } else {
      if (P->nnz == 0) HIPC(launch_fill<double>(C, P->n_user, q, ldc, 0.0, P->s));
      else {
        double *Sc = (double *)P->ucol.r;  // values permuted into column order
        HIPC(launch_gather_perm(P->nnz, P->perm, S, Sc, P->s));
        HIPC((launch_spmm<double, double>(P->ucol.pl, Sc, B, ldb, q, 1.0, nullptr, 0, 0, nullptr, 0, C, ldc,
                                 P->scratch(), P->s)));
      }
    }
    HIPC(hipStreamSynchronize(P->s));
  } catch (const BmgError &e) {
    return fail(e.st, e.msg);
  }
  return BMG_OK;
}

// ============================================================================ the method (internal orientation)
template <typename T, typename TG = T>
struct Method : Engine<T, TG> {
  using E = Engine<T, TG>;
  using E::kShadow;
  using E::P; using E::s; using E::ldk; using E::qld; using E::m; using E::n; using E::R; using E::C;
  using E::gram; using E::gemm; using E::orth; using E::z_t; using E::z_n; using E::blk; using E::avals;
  using typename E::ZOp;

  explicit Method(bmg_problem *p) : E(p) {}

  static double trace_prod(const std::vector<double> &A, const std::vector<double> &B, int k) {
    double t = 0.0;  // tr(A B) for symmetric k x k A, B
    for (size_t i = 0; i < (size_t)k * k; ++i) t += A[i] * B[i];
    return t;
  }
  double fro2(int64_t N, const T *X, int ld, int c) {
    std::vector<double> g = gram(N, c, X, ld, c, X, ld);
    double t = 0.0;
    for (int i = 0; i < c; ++i) t += g[(size_t)i * c + i];
    return t;
  }

  // ------------------------------------------------------------ BM phase
  // One preconditioned steepest-descent step with exact line search on the
  // rows-side factor (W when rows_side, else H).  Returns true if it moved.
  // polyMF-SS epoch (Sec. 6.1.1): block coordinate descent over the column
  // pairs (w_j, h_j), j = 0..k-1, from the residual of the incoming factors.
  // Per block: the direction from one pass per orientation (each pass first
  // applies the previous block's step to that orientation's stored residual),
  // the quartic's coefficients from one pass, and its exact minimiser over
  // t >= 0, found on the device so that the k blocks of an epoch run without
  // a host round trip (one fetch at the end of the epoch).  Returns whether
  // any block moved.
  bool polymf_epoch(T *W, T *H, int k, double lam) {
    if (k == 0) return false;
    double sr[2] = {0, 0}, sc[2] = {0, 0};
    const bool eg = this->exact_gather;
    this->exact_gather = true;
    if (R->pl.nnz > 0) {
      E::sddmm_store(R, W, H, k, m, n, sr);
      E::sddmm_store(C, H, W, k, n, m, sc);
    }
    this->exact_gather = eg;
    // per-row records of both sides (free during the BM phase: the gradient
    // blocks of the steepest-descent solver)
    Q4<T> *Gm = (Q4<T> *)blk(P->L.b_G), *Gn = (Q4<T> *)blk(P->L.b_D);
    double *part = (double *)P->partial;
    HIPC(launch_col_pack0<T>(m, n, W, H, ldk, Gm, Gn, s));
    // device state of the epoch: the current block's t, the number of blocks
    // that moved, a non-finite flag
    double *state = P->result + 32;
    HIPC(launch_fill<double>(state, 1, 3, 3, 0.0, s));
    for (int j = 0; j < k; ++j) {
      // from the second block on, the passes first apply the previous block's
      // step to the stored residual (a step of 0 leaves it unchanged)
      const bool upd = j > 0;
      HIPC(launch_col_grad<T>(R->pl, (T *)R->r, Gm, Gn, upd, lam, part, s));
      HIPC(launch_col_grad<T>(C->pl, (T *)C->r, Gn, Gm, upd, lam, part, s));
      E::count(R->pl, 4.0 + (upd ? 2.0 : 1.0) * sizeof(T), (double)(m + n) * 4 * sizeof(T));
      E::count(C->pl, 4.0 + (upd ? 2.0 : 1.0) * sizeof(T), (double)(m + n) * 4 * sizeof(T));
      HIPC(launch_col_quartic<T>(R->pl, (const T *)R->r, m, n, Gm, Gn, P->wsum, 2 * P->L.wsum_cap,
                                 P->wpart, P->result, lam, state, s));
      E::count(R->pl, 4.0 + sizeof(T), (double)(m + n) * 4 * sizeof(T));
      HIPC(launch_col_step<T>(m, n, W, H, ldk, j, j + 1 < k ? j + 1 : -1, state, Gm, Gn, s));
    }
    double h[3];
    E::fetch(h, state, 3);
    REQUIRE(h[2] == 0.0, BMG_ENONFINITE, "non-finite polyMF-SS line search");
    return h[1] > 0.0;
  }

  bool bm_half(bool rows_side, T *W, T *H, int k, double lam) {
    const int64_t nown = rows_side ? m : n, noth = rows_side ? n : m;
    T *own = rows_side ? W : H;
    const T *oth = rows_side ? H : W;
    T *G = blk(P->L.b_G), *D = blk(P->L.b_D);
    if (rows_side) E::grad_rows(W, H, k, lam, G);
    else E::grad_cols(W, H, k, lam, G);
    // preconditioner (oth^T oth + lam I)^{-1}
    std::vector<double> Pk = gram(noth, k, oth, ldk, k, oth, ldk);
    for (int i = 0; i < k; ++i) Pk[(size_t)i * k + i] += lam;
    std::vector<double> Pi((size_t)k * k);
    REQUIRE(lat::spd_inv(k, Pk.data(), Pi.data()), BMG_ENONFINITE, "BM preconditioner not SPD");
    std::vector<double> GG = gram(nown, k, G, ldk, k, G, ldk);
    // <G, D> = -tr(G^T G P), ||D||^2 = tr(P G^T G P)
    const double gd = trace_prod(GG, Pi, k);
    if (!(gd > 0.0)) return false;
    std::vector<double> PGGP((size_t)k * k, 0.0), tmp((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        double a = 0.0;
        for (int l = 0; l < k; ++l) a += GG[(size_t)i * k + l] * Pi[(size_t)l * k + j];
        tmp[(size_t)i * k + j] = a;
      }
    double dd = 0.0;
    for (int i = 0; i < k; ++i)
      for (int l = 0; l < k; ++l) dd += Pi[(size_t)i * k + l] * tmp[(size_t)l * k + i];
    std::vector<double> negP(Pi);
    for (double &v : negP) v = -v;
    gemm(nown, k, G, ldk, k, negP, D, ldk, 0.0);
    const double curv = rows_side ? E::curvature(R, D, oth, k, nown, noth)
                                  : E::curvature(C, D, oth, k, nown, noth);
    const double denom = curv + lam * dd;
    REQUIRE(std::isfinite(denom) && std::isfinite(gd), BMG_ENONFINITE, "non-finite BM line search");
    if (!(denom > 0.0)) return false;
    const double step = gd / denom;
    HIPC(launch_axpy<T>(nown, k, step, D, ldk, own, ldk, s));
    return true;
  }

  // F~(W, H) = f + lam/2 (||W||^2 + ||H||^2)
  double bm_objective(const T *W, const T *H, int k, double lam) {
    if (k == 0) return E::loss(W, H, 0);
    return E::loss(W, H, k) + 0.5 * lam * (fro2(m, W, ldk, k) + fro2(n, H, ldk, k));
  }

  // ------------------------------------------------------------ prox tail
  // Exact SVD of Uhat^T Z from Y = Z^T Uhat (n x q) and its Gram matrix, then
  // soft-thresholding at beta (eqs. exactSVD, approxSVD, truncate).
  struct Tail {
    int k = 0, q = 0;
    std::vector<double> sig_hat, sigma;  // all q / kept k
    bool has_u = false;
    double sum_sig2 = 0.0;
  };
  Tail prox_tail(const T *U, const T *Y, int q, const std::vector<double> &Tq, double beta, T *Wn,
                 T *Hn, T *Unew, T *uvec) {
    Tail out;
    out.q = q;
    if (q == 0) return out;
    std::vector<double> w(q), V((size_t)q * q);
    lat::sym_eig(q, Tq.data(), w.data(), V.data());
    out.sig_hat.resize(q);
    for (int j = 0; j < q; ++j) {
      out.sig_hat[j] = sqrt(std::max(w[j], 0.0));
      out.sum_sig2 += std::max(w[j], 0.0);
    }
    int k = 0;
    while (k < q && out.sig_hat[k] - beta > 0.0) ++k;
    REQUIRE(k <= P->L.k_cap, BMG_ENOMEM,
            "rank of the prox output (" + std::to_string(k) + ") exceeds k_cap");
    out.k = k;
    std::vector<double> CW((size_t)q * k), CH((size_t)q * k), CU((size_t)q * k);
    for (int j = 0; j < k; ++j) {
      const double sg = out.sig_hat[j] - beta;
      out.sigma.push_back(sg);
      const double a = sqrt(sg), b = sqrt(sg) / out.sig_hat[j];
      for (int i = 0; i < q; ++i) {
        CW[(size_t)i * k + j] = V[(size_t)i * q + j] * a;
        CH[(size_t)i * k + j] = V[(size_t)i * q + j] * b;
        CU[(size_t)i * k + j] = V[(size_t)i * q + j];
      }
    }
    gemm(m, q, U, qld, k, CW, Wn, ldk, 0.0);
    gemm(n, q, Y, qld, k, CH, Hn, ldk, 0.0);
    gemm(m, q, U, qld, k, CU, Unew, ldk, 0.0);
    if (k < q) {
      std::vector<double> cu(q);
      for (int i = 0; i < q; ++i) cu[i] = V[(size_t)i * q + k];
      gemm(m, q, U, qld, 1, cu, uvec, 1, 0.0);
      out.has_u = true;
    }
    return out;
  }

  // ------------------------------------------------------------ Algorithm 2
  // U0 (m x q0, orthonormal) in Ubuf (block B1 or B2).  On return *Uout / *Yout
  // point at the final basis (q columns) and Z^T of it; Tq is their Gram matrix.
  // History length p_t = hist_p.
  // orth([Ub, c]) for the cb orthonormal columns Ub (mm rows, ld qld) and the
  // column c right after them: c projected off ran(Ub) twice (against
  // rounding) and scaled to unit norm in place.  Returns cb + 1, or cb when
  // what is left of c is at most ORTH_TOL of its norm (the rank cut of orth()).
  // The same range as orth() of the whole block, two host round trips.
  int append_orth(int64_t mm, T *Ub, int cb) {
    T *c = Ub + cb;
    double n0 = 0.0, n1 = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      // [Ub, c]^T c: the projections and |c|^2 in one product
      std::vector<double> g = gram(mm, cb + 1, Ub, qld, 1, c, qld);
      double p2 = 0.0;
      for (int j = 0; j < cb; ++j) p2 += g[j] * g[j];
      if (pass == 0) n0 = sqrt(std::max(g[cb], 0.0));
      n1 = sqrt(std::max(g[cb] - p2, 0.0));
      if (cb > 0) {
        std::vector<double> cf(g.begin(), g.begin() + cb);
        for (double &v : cf) v = -v;
        gemm(mm, cb, Ub, qld, 1, cf, c, qld, 1.0);
      }
    }
    if (!(n0 > 0.0) || !(n1 > ORTH_TOL * n0)) return cb;
    HIPC(launch_axpy<T>(mm, 1, 1.0 / n1 - 1.0, c, qld, c, qld, s));
    return cb + 1;
  }

  // The extra column u_t + xi_t of eq. rt (Suppl. A.1.3) into col (ld qld),
  // against the cb orthonormal columns of Ub (mm rows, ld qld): u_t is u
  // projected onto ker(Ub^T) (when has_u), xi_t a standard normal vector
  // (stream STREAM_SAFEGUARD + t) projected onto ker([Ub, u_t]^T) and scaled
  // to norm psi; without u the column is that vector at norm 1.  ut and zv are
  // mm-element scratch vectors.
  void safeguard_col(int64_t mm, const T *Ub, int cb, const T *u, bool has_u, double psi,
                     uint64_t seed, int t, T *col, T *ut, T *zv) {
    HIPC(launch_normals<T>(seed, STREAM_SAFEGUARD + (uint64_t)t, mm, 1, 1, zv, s));
    double nu = 0.0;
    if (has_u) {
      HIPC(launch_copy_cols<T>(mm, 1, u, 1, ut, 1, s));
      if (cb > 0) {
        std::vector<double> c = gram(mm, cb, Ub, qld, 1, ut, 1);
        for (double &v : c) v = -v;
        gemm(mm, cb, Ub, qld, 1, c, ut, 1, 1.0);
      }
      nu = sqrt(gram(mm, 1, ut, 1, 1, ut, 1)[0]);
    }
    if (cb > 0) {
      std::vector<double> c = gram(mm, cb, Ub, qld, 1, zv, 1);
      for (double &v : c) v = -v;
      gemm(mm, cb, Ub, qld, 1, c, zv, 1, 1.0);
    }
    if (nu > 0.0) {
      const double c = gram(mm, 1, ut, 1, 1, zv, 1)[0] / (nu * nu);
      HIPC(launch_axpy<T>(mm, 1, -c, ut, 1, zv, 1, s));
    }
    const double nz = sqrt(gram(mm, 1, zv, 1, 1, zv, 1)[0]);
    const double scale = nz > 0.0 ? 1.0 / nz : 0.0;
    // column = u_t + psi * xi  (or the unit random vector when no u is kept)
    HIPC(launch_fill<T>(col, mm, 1, qld, 0.0, s));
    HIPC(launch_axpy<T>(mm, 1, (has_u ? psi : 1.0) * scale, zv, 1, col, qld, s));
    if (has_u) HIPC(launch_axpy<T>(mm, 1, 1.0, ut, 1, col, qld, s));
  }

  int hist_p = 0;
  HostHelper helper;
  int lmsvd(const ZOp &z, T *Ubuf, int q, double tau, int max_iter, double keep_level,
            T **Uout, T **Yout, std::vector<double> &Tq, int *iters) {
    if (hist_p > 0) return lmsvd_hist(z, Ubuf, q, tau, max_iter, keep_level, Uout, Yout, Tq, iters);
    T *U = Ubuf, *Y = blk(P->L.b_Y), *V = blk(P->L.b_B3), *tmp = blk(P->L.b_B4);
    z_t(z, U, q, Y);
    std::vector<double> prev;
    int it = 0;
    for (it = 1; it <= max_iter && q > 0; ++it) {
      std::vector<double> Tm = gram(n, q, Y, qld, q, Y, qld);
      // L(U) = Z Z^T U (Ritz rotation omitted: same range), queued first; the
      // Ritz values (eigenvalues of Tm, for the stopping test) are computed on
      // the helper thread while this one orthonormalises
      z_n(z, Y, q, V);
      std::vector<double> theta(q);
      double la_s = 0.0;
      {
        const int qq = q;
        helper.run([&, qq] {
          HostTimer t(la_s);
          la::sym_eig(qq, Tm.data(), theta.data(), nullptr);
        });
        HelperJoin join{helper};
        q = orth(m, V, q, U, tmp);     // U^{t,i+1}
        z_t(z, U, q, Y);
      }
      t_la_acc += la_s;
      if (ritz_converged(theta, prev, tau, keep_level)) break;
    }
    *iters = std::min(it, max_iter);
    return finish(U, Y, q, blk(P->L.b_B4), blk(P->L.b_Y2), Uout, Yout, Tq);
  }

  // stopping test: the leading Ritz values above keep_level (and the largest)
  // moved by at most tau * largest since the previous iteration
  static bool ritz_converged(const std::vector<double> &theta, std::vector<double> &prev,
                             double tau, double keep_level) {
    bool done = false;
    if (!prev.empty() && prev.size() == theta.size() && !theta.empty()) {
      double dmax = 0.0;
      for (size_t j = 0; j < theta.size(); ++j)
        if (j == 0 || theta[j] > keep_level) dmax = std::max(dmax, fabs(theta[j] - prev[j]));
      done = dmax <= tau * std::max(theta[0], 0.0);
    }
    prev = theta;
    return done;
  }

  // Algorithm 2's final cut: keep columns with s_j = ||Z^T u_j|| > eps * max
  // (selected columns go to Usel / Ysel, which must differ from U / Y)
  int finish(T *U, T *Y, int q, T *Usel, T *Ysel, T **Uout, T **Yout, std::vector<double> &Tq) {
    Tq = gram(n, q, Y, qld, q, Y, qld);
    double smax = 0.0;
    for (int j = 0; j < q; ++j) smax = std::max(smax, sqrt(std::max(Tq[(size_t)j * q + j], 0.0)));
    std::vector<int> J;
    for (int j = 0; j < q; ++j)
      if (sqrt(std::max(Tq[(size_t)j * q + j], 0.0)) > SSI_EPS * smax) J.push_back(j);
    if ((int)J.size() < q) {
      const int qj = (int)J.size();
      std::vector<double> Sel((size_t)q * qj, 0.0), Tj((size_t)qj * qj);
      for (int c = 0; c < qj; ++c) Sel[(size_t)J[c] * qj + c] = 1.0;
      gemm(m, q, U, qld, qj, Sel, Usel, qld, 0.0);
      gemm(n, q, Y, qld, qj, Sel, Ysel, qld, 0.0);
      for (int a = 0; a < qj; ++a)
        for (int b = 0; b < qj; ++b) Tj[(size_t)a * qj + b] = Tq[(size_t)J[a] * q + J[b]];
      Tq = Tj;
      U = Usel;
      Y = Ysel;
      q = qj;
    }
    *Uout = U;
    *Yout = Y;
    return q;
  }

  // The history blocks ((2p - 1) m-side and 3p n-side blocks of qld columns)
  // in the workspace region reserved at creation for p_t up to L.hist_p.
  T *hist_mem(int hp) {
    REQUIRE(hp <= P->L.hist_p, BMG_ENOMEM,
            "lmsvd_p = " + std::to_string(hp) + " needs history blocks the workspace was not sized for "
            "(it reserves p <= " + std::to_string(P->L.hist_p) + ")");
    return (T *)P->template at<char>(P->L.hist);
  }

  // Algorithm 2 with p_t = hist_p >= 1.  U^{t,i} and Z^T U^{t,i} live in a ring
  // of hist_p + 1 block pairs; the last hist_p iterates are the history.  Per
  // iteration, with U_old the history blocks and Y_old = Z^T U_old:
  //   C = U^T U_old,  P = U_old - U C (eq. PUi),  P^T P = U~ Lambda U~^T,
  //   S = U~ Lambda^{-1/2} over the eigenvalues above LMSVD_EIG_TOL (trimming),
  //   Q = [U, P S] (eq. orth-W),  Z^T Q = [Y, E] with E = (Y_old - Y C) S,
  //   L = (Z^T Q)^T (Z^T Q) = Q^T L_t(Q), V = its k_t leading eigenvectors
  //   (eq. lmsvd-opt),  Z^T Uhat = [Y, E] V,  U^{t,i+1} = orth(Z Z^T Uhat).
  // Two sparse passes per iteration, as with p_t = 0: Z^T of the basis comes
  // from products already made.
  int lmsvd_hist(const ZOp &z, T *Ubuf, int q, double tau, int max_iter, double keep_level,
                 T **Uout, T **Yout, std::vector<double> &Tq, int *iters) {
    const int hp = hist_p;
    T *B1 = blk(P->L.b_B1), *B2 = blk(P->L.b_B2);
    REQUIRE(Ubuf == B1 || Ubuf == B2, BMG_EINVAL, "subspace iteration: unexpected start block");
    char *hm = (char *)hist_mem(hp);
    const size_t mb = P->L.hist_mb, nb = P->L.hist_nb;
    std::vector<T *> Ur(hp + 1), Yr(hp + 1), Pm(hp), Bm(hp), Em(hp);
    Ur[0] = Ubuf;
    Ur[1] = Ubuf == B1 ? B2 : B1;
    Yr[0] = blk(P->L.b_Y);
    Yr[1] = blk(P->L.b_Y2);
    size_t o = 0;
    for (int j = 2; j <= hp; ++j, o += mb) Ur[j] = (T *)(hm + o);
    for (int j = 0; j < hp; ++j, o += mb) Pm[j] = (T *)(hm + o);
    for (int j = 2; j <= hp; ++j, o += nb) Yr[j] = (T *)(hm + o);
    for (int j = 0; j < hp; ++j, o += nb) Bm[j] = (T *)(hm + o);
    for (int j = 0; j < hp; ++j, o += nb) Em[j] = (T *)(hm + o);
    T *Yh = (T *)(hm + o);
    T *V = blk(P->L.b_B3), *tmp = blk(P->L.b_B4);
    int cur = 0;
    std::vector<int> hs, hw;          // ring slots and widths of the history, newest first
    z_t(z, Ur[cur], q, Yr[cur]);
    std::vector<double> prev;
    int it = 0;
    for (it = 1; it <= max_iter && q > 0; ++it) {
      T *U = Ur[cur], *Y = Yr[cur];
      const int kt = q, nh = (int)hs.size();
      int r = 0;
      std::vector<int> ew;              // widths of the column blocks of E
      std::vector<double> Lm;
      if (nh == 0) {
        Lm = gram(n, q, Y, qld, q, Y, qld);
      } else {
        std::vector<int> off(nh + 1, 0);
        for (int j = 0; j < nh; ++j) off[j + 1] = off[j] + hw[j];
        const int qo = off[nh];
        for (int j = 0; j < nh; ++j) {
          std::vector<double> negC = gram(m, q, U, qld, hw[j], Ur[hs[j]], qld);
          for (double &v : negC) v = -v;
          HIPC(launch_copy_cols<T>(m, hw[j], Ur[hs[j]], qld, Pm[j], qld, s));
          gemm(m, q, U, qld, hw[j], negC, Pm[j], qld, 1.0);      // P block j
          HIPC(launch_copy_cols<T>(n, hw[j], Yr[hs[j]], qld, Bm[j], qld, s));
          gemm(n, q, Y, qld, hw[j], negC, Bm[j], qld, 1.0);      // Z^T of P block j
        }
        std::vector<double> G((size_t)qo * qo);
        for (int a = 0; a < nh; ++a)
          for (int b = a; b < nh; ++b) {
            std::vector<double> g = gram(m, hw[a], Pm[a], qld, hw[b], Pm[b], qld);
            for (int i = 0; i < hw[a]; ++i)
              for (int j = 0; j < hw[b]; ++j) {
                G[(size_t)(off[a] + i) * qo + off[b] + j] = g[(size_t)i * hw[b] + j];
                G[(size_t)(off[b] + j) * qo + off[a] + i] = g[(size_t)i * hw[b] + j];
              }
          }
        std::vector<double> lam(qo), Ut((size_t)qo * qo);
        lat::sym_eig(qo, G.data(), lam.data(), Ut.data());
        while (r < qo && lam[r] > LMSVD_EIG_TOL) ++r;
        // E = B S in column blocks of at most qld
        for (int c0 = 0; c0 < r; c0 += qld) ew.push_back(std::min(qld, r - c0));
        for (size_t l = 0; l < ew.size(); ++l) {
          const int c0 = (int)l * qld;
          for (int j = 0; j < nh; ++j) {
            std::vector<double> Sj((size_t)hw[j] * ew[l]);
            for (int i = 0; i < hw[j]; ++i)
              for (int c = 0; c < ew[l]; ++c)
                Sj[(size_t)i * ew[l] + c] = Ut[(size_t)(off[j] + i) * qo + c0 + c] / sqrt(lam[c0 + c]);
            gemm(n, hw[j], Bm[j], qld, ew[l], Sj, Em[l], qld, j ? 1.0 : 0.0);
          }
        }
        // L = [Y, E]^T [Y, E]
        const int qq = q + r;
        Lm.assign((size_t)qq * qq, 0.0);
        auto put_block = [&](int r0, int c0, int ra, int cb, const std::vector<double> &g) {
          for (int i = 0; i < ra; ++i)
            for (int j = 0; j < cb; ++j) {
              Lm[(size_t)(r0 + i) * qq + c0 + j] = g[(size_t)i * cb + j];
              Lm[(size_t)(c0 + j) * qq + r0 + i] = g[(size_t)i * cb + j];
            }
        };
        put_block(0, 0, q, q, gram(n, q, Y, qld, q, Y, qld));
        for (size_t a = 0; a < ew.size(); ++a) {
          put_block(0, q + (int)a * qld, q, ew[a], gram(n, q, Y, qld, ew[a], Em[a], qld));
          for (size_t b = a; b < ew.size(); ++b)
            put_block(q + (int)a * qld, q + (int)b * qld, ew[a], ew[b],
                      gram(n, ew[a], Em[a], qld, ew[b], Em[b], qld));
        }
      }
      const int qq = q + r;
      std::vector<double> th(qq), Vv((size_t)qq * qq);
      lat::sym_eig(qq, Lm.data(), th.data(), Vv.data());
      std::vector<double> theta(th.begin(), th.begin() + kt);
      // Z^T Uhat = [Y, E] V(:, 1:k_t)
      {
        std::vector<double> Vt((size_t)q * kt);
        for (int i = 0; i < q; ++i)
          for (int c = 0; c < kt; ++c) Vt[(size_t)i * kt + c] = Vv[(size_t)i * qq + c];
        gemm(n, q, Y, qld, kt, Vt, Yh, qld, 0.0);
        for (size_t l = 0; l < ew.size(); ++l) {
          std::vector<double> Vl((size_t)ew[l] * kt);
          for (int i = 0; i < ew[l]; ++i)
            for (int c = 0; c < kt; ++c)
              Vl[(size_t)i * kt + c] = Vv[(size_t)(q + (int)l * qld + i) * qq + c];
          gemm(n, ew[l], Em[l], qld, kt, Vl, Yh, qld, 1.0);
        }
      }
      z_n(z, Yh, kt, V);                 // L_t(Uhat^{t,i})
      // U^{t,i+1} goes into the ring slot that leaves the history (or a free one)
      int nxt = -1;
      if (nh == hp) {
        nxt = hs.back();
      } else {
        for (int j = 0; j <= hp && nxt < 0; ++j)
          if (j != cur && std::find(hs.begin(), hs.end(), j) == hs.end()) nxt = j;
      }
      q = orth(m, V, kt, Ur[nxt], tmp);
      hs.insert(hs.begin(), cur);
      hw.insert(hw.begin(), kt);
      if ((int)hs.size() > hp) {
        hs.pop_back();
        hw.pop_back();
      }
      cur = nxt;
      z_t(z, Ur[cur], q, Yr[cur]);
      if (ritz_converged(theta, prev, tau, keep_level)) break;
    }
    *iters = std::min(it, max_iter);
    return finish(Ur[cur], Yr[cur], q, tmp, Yh, Uout, Yout, Tq);
  }

  // ------------------------------------------------------------ state of Algorithm 1
  struct State {
    T *W, *H, *Wn, *Hn, *Ucur, *Uprev, *uvec;
    int k = 0, kc = 0, kp = 0;
    int rank_cur = 0, rank_prev = 0, trunc_prev = 0;
    bool has_u = false;
    double psi = 0.1, res_prev = 1.0;
    std::vector<double> sigma;
  };
  void init_state(State &S) {
    S.W = blk(P->L.b_W); S.H = blk(P->L.b_H);
    S.Wn = blk(P->L.b_Wn); S.Hn = blk(P->L.b_Hn);
    S.Ucur = blk(P->L.b_Ucur); S.Uprev = blk(P->L.b_Uprev);
    S.uvec = blk(P->L.b_vec);
  }

  // Initialisation (Suppl. A.1.4): X_{-1} = 0, Z_{-1} = P_Omega(A), HMT range
  // finder + Nystrom for Z Z^T, then the prox tail with beta = lambda.
  void initialize(State &S, int k0, double lam, uint64_t seed) {
    ZOp z0{nullptr, nullptr, 0, -1.0, avals(R), avals(C), true};   // Z = 0 - (-1) * A
    T *B1 = blk(P->L.b_B1), *B2 = blk(P->L.b_B2), *B3 = blk(P->L.b_B3), *B4 = blk(P->L.b_B4);
    T *Y = blk(P->L.b_Y);
    k0 = std::max(1, std::min(k0, qld));
    HIPC(launch_normals<T>(seed, STREAM_SKETCH, m, k0, qld, B1, s));
    z_t(z0, B1, k0, Y);
    z_n(z0, Y, k0, B3);                                   // A_{-1} Om
    int r = orth(m, B3, k0, B2, B4);                      // Q
    int kq = 0;
    std::vector<double> Tq;
    T *Uf = B1;
    if (r > 0) {
      z_t(z0, B2, r, Y);
      z_n(z0, Y, r, B3);                                  // A Q
      std::vector<double> Cm = gram(m, r, B2, qld, r, B3, qld);   // Q^T A Q
      int r2 = orth(m, B3, r, B1, B4);                    // Q^ with A Q = Q^ R^
      std::vector<double> Rh = gram(m, r2, B1, qld, r, B3, qld);  // R^ = Q^^T A Q (r2 x r)
      // pseudo-inverse of C through its eigen-decomposition
      std::vector<double> cw(r), cv((size_t)r * r), Cp((size_t)r * r, 0.0);
      lat::sym_eig(r, Cm.data(), cw.data(), cv.data());
      for (int l = 0; l < r; ++l) {
        if (!(cw[0] > 0.0) || !(cw[l] > PINV_REL * cw[0])) continue;
        const double inv = 1.0 / cw[l];
        for (int i = 0; i < r; ++i)
          for (int j = 0; j < r; ++j) Cp[(size_t)i * r + j] += cv[(size_t)i * r + l] * inv * cv[(size_t)j * r + l];
      }
      std::vector<double> RC((size_t)r2 * r, 0.0), Mn((size_t)r2 * r2, 0.0);
      for (int i = 0; i < r2; ++i)
        for (int j = 0; j < r; ++j) {
          double a = 0.0;
          for (int l = 0; l < r; ++l) a += Rh[(size_t)i * r + l] * Cp[(size_t)l * r + j];
          RC[(size_t)i * r + j] = a;
        }
      for (int i = 0; i < r2; ++i)
        for (int j = 0; j < r2; ++j) {
          double a = 0.0;
          for (int l = 0; l < r; ++l) a += RC[(size_t)i * r + l] * Rh[(size_t)j * r + l];
          Mn[(size_t)i * r2 + j] = a;
        }
      std::vector<double> mw(r2), mv((size_t)r2 * r2);
      lat::sym_eig(r2, Mn.data(), mw.data(), mv.data());
      std::vector<int> pos;
      for (int l = 0; l < r2; ++l)
        if (mw[0] > 0.0 && mw[l] > SSI_EPS * mw[0]) pos.push_back(l);
      kq = (int)pos.size();
      std::vector<double> Sel((size_t)r2 * kq);
      for (int i = 0; i < r2; ++i)
        for (int c = 0; c < kq; ++c) Sel[(size_t)i * kq + c] = mv[(size_t)i * r2 + pos[c]];
      gemm(m, r2, B1, qld, kq, Sel, B2, qld, 0.0);       // Uhat_0 = Q^ U~
      z_t(z0, B2, kq, Y);
      Tq = gram(n, kq, Y, qld, kq, Y, qld);
      Uf = B2;
    }
    Tail tl = prox_tail(Uf, Y, kq, Tq, lam * 1.0, S.W, S.H, S.Ucur, S.uvec);
    S.k = tl.k;
    S.kc = tl.k;
    S.kp = 0;
    S.rank_cur = tl.k;
    S.rank_prev = 0;
    S.trunc_prev = tl.q - tl.k;
    S.has_u = tl.has_u;
    S.sigma = tl.sigma;
  }

  // One inexact PG step from X~ = W H^T (Algorithm 1, convex lifting phase).
  struct StepInfo {
    int q = 0, iters = 0, trials = 0;
    bool added = false;
    double residual = 0.0, eps = 0.0, alpha = 0.0;
  };

  // ------------------------------------------------------------ SpaRSA step rule
  // (Suppl., the SpaRSA variant): from the second PG step on, the step is the
  // BB step of eq. proxBB clipped to [alpha_min, alpha_max], shrunk by beta
  // until the prox output satisfies eq. back, floored at alpha_min (eq. back
  // holds there for L = 1).  Every trial restarts the subspace iteration from
  // the same warm start.
  bool sparsa = false;
  bmg_options sp_opt{};
  bool sp_have_prev = false;
  int sp_kprev = 0;
  struct SpMem {
    T *U0, *W, *H, *R, *X;
  };
  // the kept warm start (m x qld), the previous PG point (W, H at ldk), its
  // row-order residual and the sampled values of this step's X~ (nnz each):
  // the workspace region reserved at creation for the SpaRSA rule
  SpMem sparsa_mem() {
    REQUIRE(P->L.sparsa, BMG_ENOMEM,
            "the SpaRSA step rule needs state the workspace was not sized for");
    const Layout &L = P->L;
    char *b = P->template at<char>(L.sp);
    return SpMem{(T *)b, (T *)(b + L.sp_bu), (T *)(b + L.sp_bu + L.sp_bw),
                 (T *)(b + L.sp_bu + L.sp_bw + L.sp_bh),
                 (T *)(b + L.sp_bu + L.sp_bw + L.sp_bh + L.sp_br)};
  }
  // eq. proxBB read as the BB step ||dX||^2 / <dX, d grad f> between this PG
  // point X~ = W H^T and the previous one (grad f(X) - grad f(Y) = P_Omega(X - Y)
  // for (MC), so the denominator is ||R - R_prev||^2).  The numerator splits
  // over ran(Q), Q = orth(W), and its complement so that nothing cancels (the
  // three traces of eq. trace lose every digit once ||dX|| < ~1e-8 ||X||):
  //   ||dX||^2 = ||H (Q^T W)^T - H_prev (Q^T W_prev)^T||^2 + ||E H^T - E_prev H_prev^T||^2,
  // E = (I - Q Q^T) W, E_prev = (I - Q Q^T) W_prev (small; eq. trace on them).
  // Scratch: Bq (m x qld), B3, B4 (m x qld), Dn (n x qld).  R_prev is consumed.
  double bb_step(const T *W, const T *H, int k, const SpMem &sm, T *Bq, T *B3, T *B4, T *Dn) {
    const int kp = sp_kprev;
    auto three = [&](const T *W1, int l1, const T *H1, int k1, const T *W0, int l0, const T *H0, int k0) {
      double v = 0.0;
      if (k1 > 0) v += trace_prod(gram(m, k1, W1, l1, k1, W1, l1), gram(n, k1, H1, ldk, k1, H1, ldk), k1);
      if (k0 > 0) v += trace_prod(gram(m, k0, W0, l0, k0, W0, l0), gram(n, k0, H0, ldk, k0, H0, ldk), k0);
      if (k1 > 0 && k0 > 0) {
        std::vector<double> A = gram(m, k0, W0, l0, k1, W1, l1), B = gram(n, k0, H0, ldk, k1, H1, ldk);
        double c = 0.0;
        for (size_t i = 0; i < A.size(); ++i) c += A[i] * B[i];
        v -= 2.0 * c;
      }
      return v;
    };
    double num = 0.0;
    int r = 0;
    if (k > 0 && kp > 0) {
      HIPC(launch_copy_cols<T>(m, k, W, ldk, B3, qld, s));
      r = orth(m, B3, k, Bq, B4);
    }
    if (r == 0) {
      num = three(W, ldk, H, k, sm.W, ldk, sm.H, kp);
    } else {
      std::vector<double> G1 = gram(m, r, Bq, qld, k, W, ldk);       // Q^T W      (r x k)
      std::vector<double> G0 = gram(m, r, Bq, qld, kp, sm.W, ldk);   // Q^T W_prev (r x kp)
      auto tr = [](const std::vector<double> &G, int a, int b, double sg) {
        std::vector<double> t((size_t)a * b);  // sg * G^T laid out b x a
        for (int i = 0; i < a; ++i)
          for (int j = 0; j < b; ++j) t[(size_t)j * a + i] = sg * G[(size_t)i * b + j];
        return t;
      };
      gemm(n, k, H, ldk, r, tr(G1, r, k, 1.0), Dn, qld, 0.0);
      gemm(n, kp, sm.H, ldk, r, tr(G0, r, kp, -1.0), Dn, qld, 1.0);
      num = fro2(n, Dn, qld, r);
      std::vector<double> nG1(G1), nG0(G0);
      for (double &v : nG1) v = -v;
      for (double &v : nG0) v = -v;
      HIPC(launch_copy_cols<T>(m, k, W, ldk, B3, qld, s));
      gemm(m, r, Bq, qld, k, nG1, B3, qld, 1.0);                    // E
      HIPC(launch_copy_cols<T>(m, kp, sm.W, ldk, B4, qld, s));
      gemm(m, r, Bq, qld, kp, nG0, B4, qld, 1.0);                   // E_prev
      num += three(B3, qld, H, k, B4, qld, sm.H, kp);
    }
    num = std::max(num, 0.0);
    double den = 0.0;
    if (R->pl.nnz > 0) {
      HIPC(launch_axpy<T>(R->pl.nnz, 1, -1.0, (const T *)R->r, 1, sm.R, 1, s));
      den = gram(R->pl.nnz, 1, sm.R, 1, 1, sm.R, 1)[0];
    }
    const double ab = den > 0.0 ? num / den : sp_opt.alpha_max;
    return std::min(sp_opt.alpha_max, std::max(sp_opt.alpha_min, ab));
  }
  // eq. back at X+ = Wn Hn^T (rank kn) from X~:
  //   f(X+) <= f(X~) + <grad f(X~), X+ - X~> + delta / alpha ||X+ - X~||^2.
  // For the quadratic MC loss the left side minus the first two terms is
  // exactly 1/2 ||P_Omega(X+ - X~)||^2, tested in that form (the f terms nearly
  // cancel once steps are small): one sampled pass of X+ against the sampled
  // values of X~ (xs = R~ + A), with FP32 gathers in the BF16 mode.
  // d2 = ||X+ - X~||^2.
  bool back_condition(State &S, int kn, const T *xs, double d2, double alpha, double delta) {
    double lhs = 0.0;
    if (R->pl.nnz > 0) {
      const bool eg = this->exact_gather;
      this->exact_gather = true;
      lhs = E::loss_vs(xs, S.Wn, S.Hn, kn);
      this->exact_gather = eg;
    }
    return lhs <= delta / alpha * d2;
  }
  // FP64 sampled residual of both orientations from the FP32 masters (BF16
  // mode refresh): R in FP64 from FP64 copies of W, H and the FP64 values,
  // stored back in the pass type.
  void residual_fp64(const T *W, const T *H, int k, double sr[2]) {
    double *W64 = P->template at<double>(P->L.d_W64), *H64 = P->template at<double>(P->L.d_H64);
    double *R64 = P->template at<double>(P->L.d_R64);
    HIPC((launch_convert_cols<T, double>(m, k, W, ldk, W64, ldk, s)));
    HIPC((launch_convert_cols<T, double>(n, k, H, ldk, H64, ldk, s)));
    double sc[2];
    HIPC((launch_sddmm<double, double>(R->pl, R->a64, W64, ldk, H64, ldk, k, R64, E::sx(1), s)));
    E::count(R->pl, 20.0, (double)(m + n) * k * 8.0);
    E::fetch(sr, P->result, 2);
    HIPC((launch_convert<double, T>(R->pl.nnz, R64, (T *)R->r, s)));
    HIPC((launch_sddmm<double, double>(C->pl, C->a64, H64, ldk, W64, ldk, k, R64, E::sx(1), s)));
    E::count(C->pl, 20.0, (double)(m + n) * k * 8.0);
    E::fetch(sc, P->result, 2);
    HIPC((launch_convert<double, T>(C->pl.nnz, R64, (T *)C->r, s)));
  }
  double loss_fp64(const T *W, const T *H, int k) {
    if (R->pl.nnz == 0) return 0.0;
    double *W64 = P->template at<double>(P->L.d_W64), *H64 = P->template at<double>(P->L.d_H64);
    HIPC((launch_convert_cols<T, double>(m, k, W, ldk, W64, ldk, s)));
    HIPC((launch_convert_cols<T, double>(n, k, H, ldk, H64, ldk, s)));
    HIPC((launch_sddmm<double, double>(R->pl, R->a64, W64, ldk, H64, ldk, k, (double *)nullptr,
                                       E::sx(1), s)));
    E::count(R->pl, 12.0, (double)(m + n) * k * 8.0);
    double h[2];
    E::fetch(h, P->result, 2);
    return 0.5 * h[0];
  }

  StepInfo pg_step(State &S, bool changed, double lam, double alpha, double tau, int ssi_max,
                   uint64_t seed, int t, bool fp64_refresh = false) {
    StepInfo info;
    const int k = S.k;
    T *B1 = blk(P->L.b_B1), *B2 = blk(P->L.b_B2), *B4 = blk(P->L.b_B4);
    // residual of X~ stored in both orientations
    double sr[2] = {0, 0}, sc[2] = {0, 0};
    if (R->pl.nnz > 0) {
      if (kShadow && fp64_refresh && k > 0) {
        residual_fp64(S.W, S.H, k, sr);
      } else {
        E::sddmm_store(R, S.W, S.H, k, m, n, sr);
        E::sddmm_store(C, S.H, S.W, k, n, m, sc);
      }
    }
    const bool hi_before = this->exact_gather;
    this->exact_gather = kShadow && (fp64_refresh || hi_before);
    // warm start (eqs. rt0 / rt0-1): orth([U_t, W~_t]) or orth([U_t, U_{t-1}])
    const T *second = changed ? S.W : S.Uprev;
    const int c2 = changed ? k : S.kp;
    HIPC(launch_copy_cols<T>(m, S.kc, S.Ucur, ldk, B1, qld, s));
    HIPC(launch_copy_cols<T>(m, c2, second, ldk, B1 + S.kc, qld, s));
    int cb = orth(m, B1, S.kc + c2, B2, B4);
    // rank safeguard (eq. rt)
    const bool add = S.trunc_prev <= 1 || S.rank_cur == S.rank_prev || cb == 0;
    T *U0 = B2;
    int q0 = cb;
    if (add) {
      safeguard_col(m, B2, cb, S.uvec, S.has_u, S.psi, seed, t, B2 + cb,
                    blk(P->L.b_vec) + 2 * rup(m, 64), blk(P->L.b_vec) + 4 * rup(m, 64));
      q0 = append_orth(m, B2, cb);
      U0 = B2;
      info.added = true;
    }
    // step size: the fixed alpha, or the BB step of eq. proxBB (SpaRSA rule)
    double a = alpha;
    T *U0keep = nullptr, *sm_x = nullptr;
    if (sparsa) {
      SpMem sm = sparsa_mem();
      U0keep = sm.U0;
      sm_x = sm.X;
      if (R->pl.nnz > 0) {  // sampled values of X~ = R~ + A
        HIPC(launch_copy_cols<T>(R->pl.nnz, 1, (const T *)R->r, 1, sm.X, 1, s));
        HIPC(launch_axpy<T>(R->pl.nnz, 1, 1.0, avals(R), 1, sm.X, 1, s));
      }
      if (sp_have_prev)
        a = bb_step(S.W, S.H, k, sm, U0 == B1 ? B2 : B1, blk(P->L.b_B3), B4, blk(P->L.b_Y2));
      // the point of this step becomes the previous one of the next
      HIPC(launch_copy_cols<T>(m, k, S.W, ldk, sm.W, ldk, s));
      HIPC(launch_copy_cols<T>(n, k, S.H, ldk, sm.H, ldk, s));
      if (R->pl.nnz > 0) HIPC(launch_copy_cols<T>(R->pl.nnz, 1, (const T *)R->r, 1, sm.R, 1, s));
      sp_kprev = k;
      sp_have_prev = true;
      if (q0 > 0) HIPC(launch_copy_cols<T>(m, q0, U0, qld, U0keep, qld, s));
    }
    // new U_cur goes into the old U_prev buffer
    std::swap(S.Ucur, S.Uprev);
    std::swap(S.kc, S.kp);
    T *Uf = nullptr, *Yf = nullptr;
    std::vector<double> Tq;
    Tail tl;
    int q = 0;
    double d2 = 0.0, x2 = 0.0;
    if (k > 0) x2 = trace_prod(gram(m, k, S.W, ldk, k, S.W, ldk), gram(n, k, S.H, ldk, k, S.H, ldk), k);
    for (info.trials = 1;; ++info.trials) {
      if (info.trials > 1 && q0 > 0) HIPC(launch_copy_cols<T>(m, q0, U0keep, qld, U0, qld, s));
      ZOp z{S.W, S.H, k, a, (const T *)R->r, (const T *)C->r, false};
      int it = 0;
      q = lmsvd(z, U0, q0, tau, ssi_max, (a * lam) * (a * lam), &Uf, &Yf, Tq, &it);
      info.iters += it;
      tl = prox_tail(Uf, Yf, q, Tq, a * lam, S.Wn, S.Hn, S.Ucur, S.uvec);
      S.kc = tl.k;
      // ||X~ - X+|| = sqrt(||Uhat^T X~ - Uhat^T X+||^2 + ||(I - Uhat Uhat^T) X~||^2)
      d2 = 0.0;
      if (q > 0) {
        T *Dt = (Yf == blk(P->L.b_Y2)) ? blk(P->L.b_Y) : blk(P->L.b_Y2);  // n x q scratch
        std::vector<double> A1 = gram(m, k, S.W, ldk, q, Uf, qld);        // W~^T Uhat
        std::vector<double> A2 = gram(m, tl.k, S.Wn, ldk, q, Uf, qld);    // W+^T Uhat
        for (double &v : A2) v = -v;
        // Dt = H~ (W~^T Uhat) - H+ (W+^T Uhat)  =  (Uhat^T X~ - Uhat^T X+)^T
        if (k > 0) gemm(n, k, S.H, ldk, q, A1, Dt, qld, 0.0);
        else HIPC(launch_fill<T>(Dt, n, q, qld, 0.0, s));
        if (tl.k > 0) gemm(n, tl.k, S.Hn, ldk, q, A2, Dt, qld, 1.0);
        d2 = fro2(n, Dt, qld, q);
        if (k > 0) {
          T *Em = blk(P->L.b_D);
          HIPC(launch_copy_cols<T>(m, k, S.W, ldk, Em, ldk, s));
          std::vector<double> negA1(A1);
          for (double &v : negA1) v = -v;
          gemm(m, q, Uf, qld, k, [&] {  // (Uhat^T W~) laid out q x k
            std::vector<double> t2((size_t)q * k);
            for (int i = 0; i < k; ++i)
              for (int j = 0; j < q; ++j) t2[(size_t)j * k + i] = negA1[(size_t)i * q + j];
            return t2;
          }(), Em, ldk, 1.0);
          std::vector<double> EE = gram(m, k, Em, ldk, k, Em, ldk);
          std::vector<double> HH = gram(n, k, S.H, ldk, k, S.H, ldk);
          d2 += std::max(0.0, trace_prod(EE, HH, k));
        }
      } else {
        d2 = x2;
      }
      if (!sparsa || a <= sp_opt.alpha_min) break;
      if (back_condition(S, tl.k, sm_x, d2, a, sp_opt.sparsa_delta)) break;
      a = std::max(sp_opt.alpha_min, a * sp_opt.sparsa_beta);
    }
    info.q = q;
    info.alpha = a;
    info.residual = sqrt(d2) / (1.0 + sqrt(std::max(x2, 0.0)) + sqrt(sr[0]));
    const double z2 = x2 - 2.0 * a * sr[1] + a * a * sr[0];
    info.eps = sqrt(std::max(z2 - tl.sum_sig2, 0.0));
    // safeguard bookkeeping
    this->exact_gather = hi_before;
    const int trunc = tl.q - tl.k;
    S.has_u = trunc >= 1;
    if (trunc == 1) S.psi *= 0.5;
    S.trunc_prev = trunc;
    S.rank_prev = S.rank_cur;
    S.rank_cur = tl.k;
    std::swap(S.W, S.Wn);
    std::swap(S.H, S.Hn);
    S.k = tl.k;
    S.sigma = tl.sigma;
    return info;
  }

  double objective_balanced(State &S, double lam, bool fp64 = false) {
    double ssum = 0.0;
    for (double v : S.sigma) ssum += v;
    if (kShadow && fp64) return (S.k > 0 ? loss_fp64(S.W, S.H, S.k) : E::loss(S.W, S.H, 0)) + lam * ssum;
    return E::loss(S.W, S.H, S.k) + lam * ssum;
  }

  // Algorithm 1, one outer iteration per call of solve_step (so that a driver
  // can interleave several solves on one host thread)
  struct Run {
    bmg_options o{};
    State *S = nullptr;
    std::chrono::steady_clock::time_point t0;
    double F = 0.0, F_bm = 0.0, resid = INFINITY, eps = 0.0, last_refresh = INFINITY, alpha_last = 0.0;
    int every = 1, t = 0, ssi_total = 0, trials_total = 0;
    bool hi = false, conv = false, done = false;
    double la = 0.0, wait = 0.0;     // host accounting of this solve
    int syncs = 0;
  };
  // host accounting is per thread; a run carries its own across steps
  struct Acct {
    Run &r;
    explicit Acct(Run &rr) : r(rr) { t_la_acc = r.la; t_wait_acc = r.wait; n_sync_acc = r.syncs; }
    ~Acct() { r.la = t_la_acc; r.wait = t_wait_acc; r.syncs = n_sync_acc; }
  };
  void solve_begin(const bmg_options &o, State &S, Run &r) {
    r = Run();
    r.o = o;
    r.S = &S;
    r.t0 = std::chrono::steady_clock::now();
    Acct acct(r);
    hist_p = o.lmsvd_p;
    sparsa = o.step_rule == BMG_STEP_SPARSA;
    sp_opt = o;
    sp_have_prev = false;
    // polyMF-SS and SpaRSA read the stored residual entry by entry
    if (o.bm_solver == BMG_BM_POLYMF || sparsa) this->panel_on = false;
    if (hist_p > 0) hist_mem(hist_p);   // the workspace must hold them: fail early
    if (sparsa) sparsa_mem();
    init_state(S);
    S.psi = o.psi0;
    initialize(S, o.k_init, o.lambda, o.seed);
    r.F = objective_balanced(S, o.lambda, true);
    r.F_bm = r.F;
    r.every = std::max(1, o.refresh_every);
    r.alpha_last = o.alpha;
    r.done = o.max_iter <= 0;
  }
  // returns true once the solve has converged or reached max_iter
  bool solve_step(Run &r) {
    if (r.done) return true;
    Acct acct(r);
    const bmg_options &o = r.o;
    State &S = *r.S;
    const int t = r.t;
    // BF16 mode: every `every`-th iteration is a refresh: no BM phase (the
    // paper allows skipping it), R and F in FP64 and FP32 gathers in the PG
    // step, so only its residual certifies convergence.  Once a refreshed
    // residual is <= 1e-3 or stops falling, BF16 noise dominates the
    // remaining error and every later iteration runs with FP32 gathers.
    const bool refresh = !kShadow || r.hi || (t + 1) % r.every == 0;
    this->exact_gather = kShadow && r.hi;
    bool changed = false;
    for (int e = 0; e < o.bm_epochs && S.k > 0 && !(kShadow && refresh && !r.hi); ++e) {
      if (o.bm_solver == BMG_BM_POLYMF) {
        changed |= polymf_epoch(S.W, S.H, S.k, o.lambda);
      } else {
        changed |= bm_half(true, S.W, S.H, S.k, o.lambda);
        changed |= bm_half(false, S.W, S.H, S.k, o.lambda);
      }
    }
    r.F_bm = bm_objective(S.W, S.H, S.k, o.lambda);
    // FP32 passes cannot resolve Ritz values below ~1e-7 of the largest, and
    // passes gathering BF16 operands (relative rounding up to 2^-9) not below
    // ~1e-3: the subspace iteration stops at that resolution instead of
    // running into its iteration cap (refresh steps gather FP32)
    const bool bf16_gathers = kShadow && !refresh && !r.hi;
    const double floor =
        std::max(o.ssi_tol_floor, bf16_gathers ? 1e-3 : sizeof(T) == 4 ? 1e-6 : 0.0);
    const double tau = std::max(floor, std::min(1e-4, 0.1 * S.res_prev * S.res_prev));
    StepInfo st = pg_step(S, changed, o.lambda, o.alpha, tau, o.ssi_max_iter, o.seed, t, refresh);
    r.ssi_total += st.iters;
    r.trials_total += st.trials;
    r.alpha_last = st.alpha;
    r.resid = st.residual;
    r.eps = st.eps;
    r.F = objective_balanced(S, o.lambda, refresh);
    REQUIRE(std::isfinite(r.F) && std::isfinite(r.resid), BMG_ENONFINITE, "non-finite objective");
    if (o.verbose)
      fprintf(stderr,
              "[bmg] t=%d F=%.15g F_bm=%.15g res=%.3e k=%d q=%d ssi=%d eps=%.3e add=%d alpha=%.4g "
              "trials=%d\n",
              t, r.F, r.F_bm, r.resid, S.k, st.q, st.iters, r.eps, (int)st.added, st.alpha, st.trials);
    S.res_prev = r.resid;
    if (kShadow && refresh && !r.hi) {
      if (r.resid <= 1e-3 || r.resid > 0.7 * r.last_refresh) r.hi = true;
      r.last_refresh = r.resid;
    }
    r.t = t + 1;
    if (r.resid <= o.tol && refresh) r.conv = true;
    r.done = r.conv || r.t >= o.max_iter;
    return r.done;
  }
  bmg_status solve_end(Run &r, bmg_result *res) {
    Acct acct(r);
    State &S = *r.S;
    this->exact_gather = false;
    if (kShadow) r.F = objective_balanced(S, r.o.lambda, true);
    HIPC(hipStreamSynchronize(s));
    P->resolve_timing();
    if (res) {
      for (int c = 0; c < 3; ++c) {
        res->kernel_ms[c] = P->kms[c];
        res->kernel_bytes[c] = P->kbytes[c];
        res->kernel_launches[c] = P->klaunch[c];
      }
      res->host_la_seconds = t_la_acc;
      res->host_wait_seconds = t_wait_acc;
      res->host_syncs = n_sync_acc;
      res->k = S.k;
      res->iters = r.t;
      res->ssi_iters = r.ssi_total;
      res->pg_trials = r.trials_total;
      res->alpha_last = r.alpha_last;
      res->status = r.conv ? BMG_OK : BMG_NOT_CONVERGED;
      res->F = r.F;
      res->F_bm = r.F_bm;
      res->residual = r.resid;
      res->eps = r.eps;
      res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - r.t0).count();
      res->sparse_bytes = P->bytes;
      res->bf16_passes = P->bf16_passes;
      res->sparse_passes = P->passes;
    }
    return r.conv ? BMG_OK : BMG_NOT_CONVERGED;
  }
  bmg_status solve(const bmg_options &o, State &S, bmg_result *res) {
    Run r;
    solve_begin(o, S, r);
    while (!solve_step(r)) {
    }
    return solve_end(r, res);
  }
};

// ============================================================================ user <-> internal factor copies
// User W is m_user x ld (FP64), H is n_user x ld.  Internal rows side = W unless transposed.
template <typename T>
static void load_factors(bmg_problem *P, const double *W, const double *H, int k, int ld, T *Wi,
                         T *Hi) {
  const double *a = P->transposed ? H : W, *b = P->transposed ? W : H;
  const int64_t mi = P->mi(), ni = P->ni();
  const int ldk = P->L.ldk;
  if (k == 0) return;
  if constexpr (sizeof(T) == 8) {
    HIPC(launch_copy_cols<double>(mi, k, a, ld, (double *)Wi, ldk, P->s));
    HIPC(launch_copy_cols<double>(ni, k, b, ld, (double *)Hi, ldk, P->s));
  } else {
    HIPC(launch_convert_cols(mi, k, a, ld, (float *)Wi, ldk, P->s));
    HIPC(launch_convert_cols(ni, k, b, ld, (float *)Hi, ldk, P->s));
  }
}
template <typename T>
static void store_factors(bmg_problem *P, const T *Wi, const T *Hi, int k, double *W, double *H,
                          int ld) {
  double *a = P->transposed ? H : W, *b = P->transposed ? W : H;
  const int64_t mi = P->mi(), ni = P->ni();
  const int ldk = P->L.ldk;
  HIPC(launch_fill<double>(a, mi, ld, ld, 0.0, P->s));
  HIPC(launch_fill<double>(b, ni, ld, ld, 0.0, P->s));
  if (k == 0) return;
  if constexpr (sizeof(T) == 8) {
    HIPC(launch_copy_cols<double>(mi, k, (const double *)Wi, ldk, a, ld, P->s));
    HIPC(launch_copy_cols<double>(ni, k, (const double *)Hi, ldk, b, ld, P->s));
  } else {
    HIPC(launch_convert_cols(mi, k, (const float *)Wi, ldk, a, ld, P->s));
    HIPC(launch_convert_cols(ni, k, (const float *)Hi, ldk, b, ld, P->s));
  }
}

// ============================================================================ C ABI: method calls
extern "C" bmg_status bmg_bm_epochs(bmg_problem *P, double *W, double *H, int k, int ld,
                                    double lambda, int epochs, double *F_bm) {
  bmg_status st = check_factors(P, W, H, k, ld);
  if (st != BMG_OK) return st;
  try {
    Method<double> M(P);
    double *Wi = M.blk(P->L.b_W), *Hi = M.blk(P->L.b_H);
    load_factors<double>(P, W, H, k, ld, Wi, Hi);
    for (int e = 0; e < epochs && k > 0; ++e) {
      M.bm_half(true, Wi, Hi, k, lambda);
      M.bm_half(false, Wi, Hi, k, lambda);
    }
    if (F_bm) *F_bm = M.bm_objective(Wi, Hi, k, lambda);
    if (k > 0) {
      const double *a = P->transposed ? Hi : Wi, *b = P->transposed ? Wi : Hi;
      HIPC(launch_copy_cols<double>(P->m_user, k, a, P->L.ldk, W, ld, P->s));
      HIPC(launch_copy_cols<double>(P->n_user, k, b, P->L.ldk, H, ld, P->s));
    }
    HIPC(hipStreamSynchronize(P->s));
  } catch (const BmgError &e) {
    return fail(e.st, e.msg);
  }
  return BMG_OK;
}

extern "C" bmg_status bmg_polymf_epochs(bmg_problem *P, double *W, double *H, int k, int ld,
                                        double lambda, int epochs, double *F_bm) {
  bmg_status st = check_factors(P, W, H, k, ld);
  if (st != BMG_OK) return st;
  if (epochs < 0 || !(lambda > 0.0)) return fail(BMG_EINVAL, "bmg_polymf_epochs: bad arguments");
  try {
    Method<double> M(P);
    M.panel_on = false;   // polyMF-SS reads the stored residual entry by entry
    double *Wi = M.blk(P->L.b_W), *Hi = M.blk(P->L.b_H);
    load_factors<double>(P, W, H, k, ld, Wi, Hi);
    for (int e = 0; e < epochs && k > 0; ++e) M.polymf_epoch(Wi, Hi, k, lambda);
    if (F_bm) *F_bm = M.bm_objective(Wi, Hi, k, lambda);
    if (k > 0) {
      const double *a = P->transposed ? Hi : Wi, *b = P->transposed ? Wi : Hi;
      HIPC(launch_copy_cols<double>(P->m_user, k, a, P->L.ldk, W, ld, P->s));
      HIPC(launch_copy_cols<double>(P->n_user, k, b, P->L.ldk, H, ld, P->s));
    }
    HIPC(hipStreamSynchronize(P->s));
  } catch (const BmgError &e) {
    return fail(e.st, e.msg);
  }
  return BMG_OK;
}

extern "C" bmg_status bmg_objective(bmg_problem *P, const double *W, const double *H, int k, int ld,
                                    double lambda, double *F, double *residual) {
  bmg_status st = check_factors(P, W, H, k, ld);
  if (st != BMG_OK) return st;
  if (residual && !(lambda > 0.0)) return fail(BMG_EINVAL, "bmg_objective: the residual needs lambda > 0");
  try {
    Method<double> M(P);
    double *Wi = M.blk(P->L.b_W), *Hi = M.blk(P->L.b_H);
    load_factors<double>(P, W, H, k, ld, Wi, Hi);
    double f = M.loss(Wi, Hi, k), nuc = 0.0;
    if (k > 0) {
      // ||W H^T||_* = sum sqrt(eig(S (H^T H) S^T)) with S^T S = W^T W
      std::vector<double> WW = M.gram(M.m, k, Wi, P->L.ldk, k, Wi, P->L.ldk);
      std::vector<double> HH = M.gram(M.n, k, Hi, P->L.ldk, k, Hi, P->L.ldk);
      std::vector<double> w(k), V((size_t)k * k), Sm((size_t)k * k), T1((size_t)k * k), T2((size_t)k * k);
      lat::sym_eig(k, WW.data(), w.data(), V.data());
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) Sm[(size_t)i * k + j] = sqrt(std::max(w[i], 0.0)) * V[(size_t)j * k + i];
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
          double a = 0.0;
          for (int l = 0; l < k; ++l) a += Sm[(size_t)i * k + l] * HH[(size_t)l * k + j];
          T1[(size_t)i * k + j] = a;
        }
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
          double a = 0.0;
          for (int l = 0; l < k; ++l) a += T1[(size_t)i * k + l] * Sm[(size_t)j * k + l];
          T2[(size_t)i * k + j] = a;
        }
      lat::sym_eig(k, T2.data(), w.data(), nullptr);
      for (int i = 0; i < k; ++i) nuc += sqrt(std::max(w[i], 0.0));
    }
    if (F) *F = f + lambda * nuc;
    if (residual) {
      // one inexact PG step from X~ = W H^T at the default step and subspace
      // settings, warm-started from W alone (as bmg_prox_step); its output stays
      // in the workspace, the caller's factors are not touched
      bmg_options o;
      bmg_options_default(&o);
      Method<double>::State S;
      M.init_state(S);
      S.k = k; S.kc = 0; S.kp = 0;
      S.rank_cur = 0; S.rank_prev = 0; S.trunc_prev = 0;
      S.has_u = false;
      S.psi = o.psi0;
      auto info = M.pg_step(S, true, lambda, o.alpha, o.ssi_tol_floor, o.ssi_max_iter, o.seed, 0);
      HIPC(hipStreamSynchronize(P->s));
      *residual = info.residual;
    }
  } catch (const BmgError &e) {
    return fail(e.st, e.msg);
  }
  return BMG_OK;
}

// ============================================================================ kernel-estimation QSDP
// BM-Global for min f(X) + lambda tr(X) over {X psd, <E, X> = 0} with
// f(X) = 1/2 sum over pairs (X_ii + X_jj - 2 X_ij - d_ij^2)^2 (QSDP section), in
// the BM form X = W W^T, W^T e = 0 (eq. bm2).  Omega is stored symmetrically,
// so sums over stored entries count every pair twice.  FP64.
struct RkeMethod : Method<double> {
  using M = Method<double>;
  using M::P; using M::s; using M::ldk; using M::qld; using M::n; using M::R;
  using M::gram; using M::gemm; using M::orth; using M::blk; using M::fro2;
  explicit RkeMethod(bmg_problem *p) : M(p) {
    this->panel_on = false;
    const int64_t nv = rup(n, 64);
    deg = blk(P->L.b_vec) + 2 * nv;
    adeg = blk(P->L.b_vec) + 3 * nv;
  }
  double *deg, *adeg;

  // r (stored, CSR order) = ||w_i - w_j||^2 - d_ij^2, deg / adeg per row;
  // returns sum over stored entries of r^2
  double residual(const double *W, int k, bool fetch_sum = true) {
    HIPC(launch_rke_res(R->pl, W, ldk, k, (const double *)R->a64, (double *)R->r, deg, adeg,
                        (double *)P->partial, P->wsum, 2 * P->L.wsum_cap, P->result, s));
    E::count(R->pl, 4.0 + 16.0, (double)n * k * 8.0);
    if (!fetch_sum) return 0.0;
    double h[1];
    E::fetch(h, P->result, 1);
    return h[0];
  }
  // Frobenius inner products of up to four pairs of n x k blocks (ld ldk) into
  // P->result + off (device; fetched by the caller)
  void dots(std::initializer_list<std::pair<const double *, const double *>> pr, int k, int off) {
    const double *A[4], *B[4];
    int np = 0;
    for (auto &q : pr) {
      A[np] = q.first;
      B[np] = q.second;
      ++np;
    }
    HIPC(launch_frob_dots(n, k, ldk, A, B, np, P->wpart, P->result + off, s));
  }
  // out (ld ldo) = L_r U: the sparse x dense pass with the stored r, then deg U - (.)
  void lap(const double *U, int q, int ldu, double *out, int ldo) {
    if (q == 0) return;
    E::template pass<double>(2, R->pl, (const double *)R->r, (const double *)nullptr, ldk, U, ldu, q, 0.0,
                             1.0, out, ldo, 0, nullptr, 0, E::sx(2));
    E::count(R->pl, 4.0 + 8.0, (double)n * q * 16.0);
    HIPC(launch_rowscale_sub(n, q, deg, U, ldu, out, ldo, s));
  }
  // Y = M U with M = W W^T - alpha L_r - alpha lambda J (U^T e = 0: J U = U)
  void apply_M(const double *W, int k, double alpha, double lam, const double *U, int q, double *Y,
               double *tmp) {
    lap(U, q, qld, tmp, qld);
    if (k > 0) {
      std::vector<double> G = gram(n, k, W, ldk, q, U, qld);
      gemm(n, k, W, ldk, q, G, Y, qld, 0.0);
    } else {
      HIPC(launch_fill<double>(Y, n, q, qld, 0.0, s));
    }
    HIPC(launch_axpy<double>(n, q, -alpha, tmp, qld, Y, qld, s));
    HIPC(launch_axpy<double>(n, q, -alpha * lam, U, qld, Y, qld, s));
  }
  double dot(const double *A, const double *B, int k) {
    std::vector<double> g = gram(n, k, A, ldk, k, B, ldk);
    double t = 0.0;
    for (int i = 0; i < k; ++i) t += g[(size_t)i * k + i];
    return t;
  }
  // BM phase: `steps` nonlinear CG steps (Polak-Ribiere, restart at negative
  // beta or a non-descent direction) with the exact quartic line search.  Two
  // host round trips per step: <G, G>, <G, G_prev>, <D_prev, G> (for beta and
  // the descent test), then the quartic sums with <W, D>, <D, D>.
  void bm_phase(double *W, int k, double lam, int steps) {
    double *G = blk(P->L.b_G), *D = blk(P->L.b_D), *Gp = blk(P->L.b_H);
    double gp2 = 0.0;
    for (int st = 0; st < steps; ++st) {
      residual(W, k, false);
      lap(W, k, ldk, G, ldk);
      HIPC(launch_axpy<double>(n, k, lam, W, ldk, G, ldk, s));
      HIPC(launch_center_cols(n, k, G, ldk, P->gram_part, P->L.gram_cap, s));
      double h1[3] = {0.0, 0.0, 0.0};
      if (st == 0) {
        dots({{G, G}}, k, 0);
        E::fetch(h1, P->result, 1);
      } else {
        dots({{G, G}, {G, Gp}, {D, G}}, k, 0);
        E::fetch(h1, P->result, 3);
      }
      const double g2 = h1[0];
      bool sd = st == 0;
      if (!sd) {
        const double beta = std::max(0.0, (g2 - h1[1]) / gp2);
        // <beta D_prev - G, G> >= 0: not a descent direction, restart
        if (beta * h1[2] - g2 >= 0.0) {
          sd = true;
        } else {
          HIPC(launch_axpy<double>(n, k, beta - 1.0, D, ldk, D, ldk, s));   // D = beta D
          HIPC(launch_axpy<double>(n, k, -1.0, G, ldk, D, ldk, s));          // D -= G
        }
      }
      if (sd) {
        HIPC(launch_fill<double>(D, n, k, ldk, 0.0, s));
        HIPC(launch_axpy<double>(n, k, -1.0, G, ldk, D, ldk, s));
      }
      HIPC(launch_rke_quartic(R->pl, W, D, ldk, k, (const double *)R->r, P->wsum, 2 * P->L.wsum_cap,
                              P->result, s));
      E::count(R->pl, 4.0 + 8.0, (double)n * k * 16.0);
      dots({{W, D}, {D, D}}, k, 8);
      double h[10];
      E::fetch(h, P->result, 10);
      const double c1 = h[0] + 2.0 * lam * h[8];
      const double c2 = h[1] + 0.5 * h[2] + lam * h[9];
      const double c3 = h[3], c4 = 0.25 * h[4];
      REQUIRE(std::isfinite(c1) && std::isfinite(c2) && std::isfinite(c3) && std::isfinite(c4),
              BMG_ENONFINITE, "non-finite line search");
      const double t = quartic_min(c1, c2, c3, c4);
      if (t > 0.0) HIPC(launch_axpy<double>(n, k, t, D, ldk, W, ldk, s));
      HIPC(launch_copy_cols<double>(n, k, G, ldk, Gp, ldk, s));
      gp2 = g2;
    }
  }
  // ||W1 W1^T - W0 W0^T||_F^2 split over ran(orth(W1)) and its complement
  double diff2(const double *W1, int k1, const double *W0, int k0) {
    auto three = [&](const double *A, int la, int ka, const double *B, int lb, int kb) {
      double v = 0.0;
      if (ka > 0) { auto g = gram(n, ka, A, la, ka, A, la); v += M::trace_prod(g, g, ka); }
      if (kb > 0) { auto g = gram(n, kb, B, lb, kb, B, lb); v += M::trace_prod(g, g, kb); }
      if (ka > 0 && kb > 0) {
        auto g = gram(n, kb, B, lb, ka, A, la);
        double c = 0.0;
        for (double x : g) c += x * x;
        v -= 2.0 * c;
      }
      return v;
    };
    double *Q = blk(P->L.b_B3), *T1 = blk(P->L.b_B4), *E1 = blk(P->L.b_Y), *E0 = blk(P->L.b_Y2);
    int r = 0;
    if (k1 > 0 && k0 > 0) {
      HIPC(launch_copy_cols<double>(n, k1, W1, ldk, E1, qld, s));
      r = orth(n, E1, k1, Q, T1);
    }
    if (r == 0) return std::max(0.0, three(W1, ldk, k1, W0, ldk, k0));
    std::vector<double> G1 = gram(n, r, Q, qld, k1, W1, ldk), G0 = gram(n, r, Q, qld, k0, W0, ldk);
    // (Q^T W1)(Q^T W1)^T - (Q^T W0)(Q^T W0)^T on the host (r x r)
    double d = 0.0;
    for (int a = 0; a < r; ++a)
      for (int b = 0; b < r; ++b) {
        double v = 0.0;
        for (int c = 0; c < k1; ++c) v += G1[(size_t)a * k1 + c] * G1[(size_t)b * k1 + c];
        for (int c = 0; c < k0; ++c) v -= G0[(size_t)a * k0 + c] * G0[(size_t)b * k0 + c];
        d += v * v;
      }
    // cross term 2 ||Q^T (W1 W1^T - W0 W0^T) (I - QQ^T)||^2 = 2 ||(Q^T W0) E0^T||^2 (E1 = 0 up to rounding)
    for (double &v : G1) v = -v;
    for (double &v : G0) v = -v;
    HIPC(launch_copy_cols<double>(n, k1, W1, ldk, E1, qld, s));
    gemm(n, r, Q, qld, k1, G1, E1, qld, 1.0);
    HIPC(launch_copy_cols<double>(n, k0, W0, ldk, E0, qld, s));
    gemm(n, r, Q, qld, k0, G0, E0, qld, 1.0);
    for (double &v : G1) v = -v;
    for (double &v : G0) v = -v;
    // Q^T X E^T blocks: (Q^T W1) (E1^T) - (Q^T W0)(E0^T): Frobenius^2 via Gram matrices
    double cross = 0.0;
    {
      auto e11 = gram(n, k1, E1, qld, k1, E1, qld), e00 = gram(n, k0, E0, qld, k0, E0, qld);
      auto e01 = gram(n, k0, E0, qld, k1, E1, qld);
      auto g11 = std::vector<double>((size_t)k1 * k1), g00 = std::vector<double>((size_t)k0 * k0),
           g01 = std::vector<double>((size_t)k0 * k1);
      for (int a = 0; a < k1; ++a)
        for (int b = 0; b < k1; ++b) {
          double v = 0.0;
          for (int c = 0; c < r; ++c) v += G1[(size_t)c * k1 + a] * G1[(size_t)c * k1 + b];
          g11[(size_t)a * k1 + b] = v;
        }
      for (int a = 0; a < k0; ++a)
        for (int b = 0; b < k0; ++b) {
          double v = 0.0;
          for (int c = 0; c < r; ++c) v += G0[(size_t)c * k0 + a] * G0[(size_t)c * k0 + b];
          g00[(size_t)a * k0 + b] = v;
        }
      for (int a = 0; a < k0; ++a)
        for (int b = 0; b < k1; ++b) {
          double v = 0.0;
          for (int c = 0; c < r; ++c) v += G0[(size_t)c * k0 + a] * G1[(size_t)c * k1 + b];
          g01[(size_t)a * k1 + b] = v;
        }
      double c = 0.0;
      for (size_t i = 0; i < g11.size(); ++i) c += g11[i] * e11[i];
      for (size_t i = 0; i < g00.size(); ++i) c += g00[i] * e00[i];
      for (size_t i = 0; i < g01.size(); ++i) c -= 2.0 * g01[i] * e01[i];
      cross = std::max(0.0, c);
    }
    return d + 2.0 * cross + std::max(0.0, three(E1, qld, k1, E0, qld, k0));
  }
  struct Eig {
    int k = 0, iters = 0, q = 0;  // rank kept, iterations, Ritz values in the last basis
    bool has_u = false;           // uvec holds the Ritz vector of the largest one not kept
  };
  // Prox of the PG step (Lemma PiX) from the q0 columns of U0 (block B1 or
  // B2, ld qld): Algorithm 2 with history hp (0 or 1) on M + sigma I.  Per
  // iteration, U (q columns) and Y = M U in the first columns of their blocks;
  // with history, U_old / Y_old the previous ones:
  //   C = U^T U_old, P = U_old - U C (eq. PUi), P^T P = U~ Lambda U~^T,
  //   S = U~ Lambda^{-1/2} over the eigenvalues above LMSVD_EIG_TOL,
  //   Q = [U, P S] (eq. orth-W; P S in U's block after its q columns),
  //   M Q = [Y, (Y_old - Y C) S] (likewise in Y's block),
  //   theta, V = the q leading eigenpairs of Q^T M Q (eq. lmsvd-opt),
  //   next U = orth(J (M Q V + sigma Q V)), Y = M U.
  // Stop once the Ritz values above 0, the largest and the first one not above
  // 0 moved by at most tau * |largest|; with history (hp > 0) the newest of
  // them by at most max(tau |largest|, min(tau_new, 1e-4 |largest|)) (tau_new
  // an absolute tolerance, 0 for none).  The positive Ritz pairs of the last
  // step are kept: Wn = Q V_+ sqrt(theta_+), Uc = Q V_+ (ld ldk); uvec =
  // Q v_{k+1} when a Ritz value is not kept.
  Eig eig_prox(const double *W, int k, double alpha, double lam, double *U0, int q0, double tau,
               double tau_new, int max_iter, int hp, double *Wn, double *Uc, double *uvec) {
    Eig out;
    double *B1 = blk(P->L.b_B1), *B2 = blk(P->L.b_B2), *B3 = blk(P->L.b_B3), *B4 = blk(P->L.b_B4);
    double *Y = blk(P->L.b_Y), *tmp = blk(P->L.b_Y2);
    double *U = U0 == B1 ? B2 : B1;
    double *Uold = nullptr, *Yold = nullptr, *Pt = nullptr, *Et = nullptr;
    if (hp > 0) {
      char *hm = (char *)this->hist_mem(hp);
      const size_t mb = P->L.hist_mb, nb = P->L.hist_nb;
      Uold = (double *)hm;
      Yold = (double *)(hm + mb);
      Pt = (double *)(hm + mb + nb);
      Et = (double *)(hm + mb + 2 * nb);
    }
    // sigma = alpha (2 max_i sum_j |r_ij| + lambda)
    std::vector<double> ad(n);
    HIPC(hipMemcpyAsync(ad.data(), adeg, 8 * n, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    double amax = 0.0;
    for (double v : ad) amax = std::max(amax, v);
    const double sigma = alpha * (2.0 * amax + lam);
    HIPC(launch_center_cols(n, q0, U0, qld, P->gram_part, P->L.gram_cap, s));
    int q = orth(n, U0, q0, U, B4);
    if (q == 0) return out;
    apply_M(W, k, alpha, lam, U, q, Y, tmp);
    std::vector<double> prev, th, V;
    int qo = 0, qq = q;   // history columns, columns of Q
    int it = 0;
    for (it = 1; it <= max_iter; ++it) {
      qq = q;
      if (qo > 0) {
        std::vector<double> Cm = gram(n, q, U, qld, qo, Uold, qld);   // q x qo
        for (double &v : Cm) v = -v;
        HIPC(launch_copy_cols<double>(n, qo, Uold, qld, Pt, qld, s));
        gemm(n, q, U, qld, qo, Cm, Pt, qld, 1.0);
        std::vector<double> G = gram(n, qo, Pt, qld, qo, Pt, qld), lp(qo), Ut((size_t)qo * qo);
        lat::sym_eig(qo, G.data(), lp.data(), Ut.data());
        int r2 = 0;
        while (r2 < qo && lp[r2] > LMSVD_EIG_TOL) ++r2;
        REQUIRE(q + r2 <= qld, BMG_ENOMEM, "subspace basis wider than the workspace blocks");
        if (r2 > 0) {
          std::vector<double> Sm((size_t)qo * r2);
          for (int a = 0; a < qo; ++a)
            for (int c = 0; c < r2; ++c) Sm[(size_t)a * r2 + c] = Ut[(size_t)a * qo + c] / sqrt(lp[c]);
          gemm(n, qo, Pt, qld, r2, Sm, U + q, qld, 0.0);
          HIPC(launch_copy_cols<double>(n, qo, Yold, qld, Et, qld, s));
          gemm(n, q, Y, qld, qo, Cm, Et, qld, 1.0);
          gemm(n, qo, Et, qld, r2, Sm, Y + q, qld, 0.0);
          qq = q + r2;
        }
      }
      std::vector<double> T = gram(n, qq, U, qld, qq, Y, qld);
      for (int a = 0; a < qq; ++a)
        for (int b = 0; b < a; ++b) {
          const double v = 0.5 * (T[(size_t)a * qq + b] + T[(size_t)b * qq + a]);
          T[(size_t)a * qq + b] = T[(size_t)b * qq + a] = v;
        }
      std::vector<double> thq(qq), Vq((size_t)qq * qq);
      lat::sym_eig(qq, T.data(), thq.data(), Vq.data());
      th.assign(thq.begin(), thq.begin() + q);
      V.assign((size_t)qq * q, 0.0);
      for (int a = 0; a < qq; ++a)
        for (int c = 0; c < q; ++c) V[(size_t)a * q + c] = Vq[(size_t)a * qq + c];
      bool done = false;
      if (!prev.empty() && prev.size() == th.size()) {
        // the Ritz values kept, the largest, and the first one not kept
        int npos = 0;
        while (npos < q && th[npos] > 0.0) ++npos;
        // with history, the newest of them (the smallest kept when all are
        // kept, else the first not kept) is held to tau_new instead when that
        // is looser
        const int jn = std::min(npos, q - 1);
        const bool rel = hp > 0 && tau_new > 0.0 && jn > 0;
        double dmax = 0.0, dnew = 0.0;
        for (int j = 0; j < q; ++j)
          if (j == 0 || th[j] > 0.0 || j == jn) {
            if (rel && j == jn) dnew = fabs(th[j] - prev[j]);
            else dmax = std::max(dmax, fabs(th[j] - prev[j]));
          }
        const double lim = tau * fabs(th[0]);
        done = dmax <= lim && dnew <= std::max(lim, std::min(tau_new, 1e-4 * fabs(th[0])));
      }
      prev = th;
      if (done || it == max_iter) break;
      // next basis: orth(J (M Q V + sigma Q V))
      std::vector<double> sV(V);
      for (double &v : sV) v *= sigma;
      gemm(n, qq, Y, qld, q, V, B3, qld, 0.0);
      gemm(n, qq, U, qld, q, sV, B3, qld, 1.0);
      HIPC(launch_center_cols(n, q, B3, qld, P->gram_part, P->L.gram_cap, s));
      if (hp > 0) {
        HIPC(launch_copy_cols<double>(n, q, U, qld, Uold, qld, s));
        HIPC(launch_copy_cols<double>(n, q, Y, qld, Yold, qld, s));
        qo = q;
      }
      const int qn = orth(n, B3, q, U, B4);
      if (qn == 0) {
        out.iters = it;
        return out;
      }
      q = qn;
      apply_M(W, k, alpha, lam, U, q, Y, tmp);
    }
    out.iters = std::min(it, max_iter);
    out.q = q;
    int kp = 0;
    while (kp < q && th[kp] > 0.0) ++kp;
    REQUIRE(kp <= P->L.k_cap, BMG_ENOMEM, "rank of the prox output (" + std::to_string(kp) + ") exceeds k_cap");
    std::vector<double> CW((size_t)qq * std::max(kp, 1)), CU((size_t)qq * std::max(kp, 1));
    for (int i = 0; i < qq; ++i)
      for (int j = 0; j < kp; ++j) {
        CU[(size_t)i * kp + j] = V[(size_t)i * q + j];
        CW[(size_t)i * kp + j] = V[(size_t)i * q + j] * sqrt(th[j]);
      }
    if (kp > 0) {
      gemm(n, qq, U, qld, kp, CW, Wn, ldk, 0.0);
      gemm(n, qq, U, qld, kp, CU, Uc, ldk, 0.0);
    }
    if (kp < q) {
      std::vector<double> cu(qq);
      for (int i = 0; i < qq; ++i) cu[i] = V[(size_t)i * q + kp];
      gemm(n, qq, U, qld, 1, cu, uvec, 1, 0.0);
      out.has_u = true;
    }
    out.k = kp;
    return out;
  }

  // Algorithm 1 on the QSDP: BM phase, then the PG step of Lemma PiX with
  // step alpha / (2 + 2 max degree), warm-started from [orth(J W~), u_t + xi_t]
  // (the rank safeguard column of eq. rt, psi halving after every step that
  // truncates exactly one Ritz value); the stop residual is the PG step's
  // change divided by the step size
  bmg_status solve(const bmg_options &o, int *k_out, bmg_result *res) {
    const auto t0 = std::chrono::steady_clock::now();
    P->reset_stats();
    REQUIRE(o.lmsvd_p >= 0 && o.lmsvd_p <= 1, BMG_EINVAL,
            "the kernel-estimation path runs Algorithm 2 with lmsvd_p 0 or 1");
    const int hp = o.lmsvd_p;
    std::vector<int64_t> ptr(n + 1);
    HIPC(hipMemcpyAsync(ptr.data(), R->pl.ptr, 8 * (n + 1), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    int64_t maxdeg = 0;
    for (int64_t i = 0; i < n; ++i) maxdeg = std::max(maxdeg, ptr[i + 1] - ptr[i]);
    const double alpha = o.alpha / (2.0 + 2.0 * (double)maxdeg);
    const double lam = o.lambda;
    double *W = blk(P->L.b_W), *Wn = blk(P->L.b_Wn), *Uc = blk(P->L.b_Ucur);
    double *B1 = blk(P->L.b_B1), *B2 = blk(P->L.b_B2), *B4 = blk(P->L.b_B4);
    const int64_t nv = rup(n, 64);
    double *uvec = blk(P->L.b_vec), *ut = blk(P->L.b_vec) + 4 * nv, *zv = blk(P->L.b_vec) + 5 * nv;
    int k = 0, ssi_total = 0;
    // X_{-1} = 0: r = -d^2; the start block J times Gaussian (n x k0)
    const int k0 = std::max(1, std::min(o.k_init, qld));
    residual(W, 0);
    HIPC(launch_normals<double>(o.seed, STREAM_SKETCH, n, k0, qld, B1, s));
    Eig e0 = eig_prox(W, 0, alpha, lam, B1, k0, 1e-4, 0.0, o.ssi_max_iter, hp, Wn, Uc, uvec);
    ssi_total += e0.iters;
    k = e0.k;
    bool has_u = e0.has_u;
    double psi = o.psi0;
    std::swap(W, Wn);
    double resid = INFINITY, res_prev = 1.0, F = 0.0, step_prev = 0.0;
    bool conv = false;
    int t = 0;
    for (t = 0; t < o.max_iter; ++t) {
      if (k > 0 && o.bm_epochs > 0) bm_phase(W, k, lam, o.bm_epochs);
      const double r2 = residual(W, k);
      const double tau = std::max(o.ssi_tol_floor, std::min(1e-4, 0.1 * res_prev * res_prev));
      // warm start [orth(J W~_t), u_t + xi_t]: the rank grows by at most one per step
      int cb = 0;
      if (k > 0) {
        HIPC(launch_copy_cols<double>(n, k, W, ldk, B1, qld, s));
        HIPC(launch_center_cols(n, k, B1, qld, P->gram_part, P->L.gram_cap, s));
        cb = orth(n, B1, k, B2, B4);
      }
      this->safeguard_col(n, B2, cb, uvec, has_u, psi, o.seed, t, B2 + cb, ut, zv);
      // the newest Ritz value's tolerance: a tenth of the previous PG step
      Eig ep = eig_prox(W, k, alpha, lam, B2, cb + 1, tau, 0.1 * step_prev, o.ssi_max_iter, hp, Wn, Uc,
                        uvec);
      ssi_total += ep.iters;
      // safeguard bookkeeping (eq. rt)
      const int trunc = ep.q - ep.k;
      has_u = ep.has_u && trunc >= 1;
      if (trunc == 1) psi *= 0.5;
      // relative residual ||X~ - X+|| / (1 + ||X~|| + ||grad f~(X~)||)
      std::vector<double> dg(n);
      HIPC(hipMemcpyAsync(dg.data(), deg, 8 * n, hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      double g2 = r2;
      for (double v : dg) g2 += (v + lam) * (v + lam);
      double x2 = 0.0;
      if (k > 0) { auto g = gram(n, k, W, ldk, k, W, ldk); x2 = M::trace_prod(g, g, k); }
      const double d2 = k > 0 ? diff2(W, k, Wn, ep.k)
                              : (ep.k > 0 ? [&] { auto g = gram(n, ep.k, Wn, ldk, ep.k, Wn, ldk);
                                                  return M::trace_prod(g, g, ep.k); }() : 0.0);
      // the prox-gradient mapping (divided by alpha, which is far below 1 here)
      resid = sqrt(std::max(d2, 0.0)) / (alpha * (1.0 + sqrt(std::max(x2, 0.0)) + sqrt(g2)));
      step_prev = sqrt(std::max(d2, 0.0));
      std::swap(W, Wn);
      k = ep.k;
      F = 0.25 * residual(W, k) + lam * (k > 0 ? fro2(n, W, ldk, k) : 0.0);
      REQUIRE(std::isfinite(F) && std::isfinite(resid), BMG_ENONFINITE, "non-finite objective");
      if (o.verbose)
        fprintf(stderr, "[bmg-rke] t=%d F=%.15g res=%.3e k=%d ssi=%d\n", t, F, resid, k, ep.iters);
      res_prev = resid;
      if (resid <= o.tol) {
        conv = true;
        ++t;
        break;
      }
    }
    HIPC(hipStreamSynchronize(s));
    last_W = W;
    *k_out = k;
    if (res) {
      memset(res, 0, sizeof(*res));
      res->k = k;
      res->iters = t;
      res->ssi_iters = ssi_total;
      res->status = conv ? BMG_OK : BMG_NOT_CONVERGED;
      res->F = F;
      res->residual = resid;
      res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      res->sparse_bytes = P->bytes;
      res->sparse_passes = P->passes;
    }
    return conv ? BMG_OK : BMG_NOT_CONVERGED;
  }
  double *last_W = nullptr;
};

static bmg_status check_rke(bmg_problem *P) {
  if (!P) return fail(BMG_EINVAL, "null problem");
  if (P->prec != BMG_FP64) return fail(BMG_EINVAL, "the kernel-estimation path runs in BMG_FP64");
  if (P->m_user != P->n_user) return fail(BMG_EINVAL, "the kernel-estimation path needs a square Omega");
  try {
    RkeMethod M(P);
    int *flag = (int *)P->result;
    HIPC(hipMemsetAsync(flag, 0, sizeof(int), P->s));
    HIPC(launch_cmp_orient(M.R->pl.nnz, M.R->pl.idx, M.C->pl.idx, M.R->a64, M.C->a64, flag, P->s));
    int h = 0;
    HIPC(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, P->s));
    HIPC(hipStreamSynchronize(P->s));
    if (h) return fail(BMG_EINVAL, "Omega and its values must be symmetric (both (i, j) and (j, i) stored)");
  } catch (const BmgError &e) {
    return fail(e.st, e.msg);
  }
  return BMG_OK;
}

extern "C" bmg_status bmg_rke_residual(bmg_problem *P, const double *W, int k, int ld, double *r,
                                       double *deg, double *sumsq) {
  bmg_status st = check_rke(P);
  if (st != BMG_OK) return st;
  if (k < 0 || k > P->L.k_cap || ld < k || ld % 8 != 0 || (k > 0 && !W))
    return fail(BMG_EINVAL, "bad k / ld");
  try {
    RkeMethod M(P);
    double *Wi = M.blk(P->L.b_W);
    if (k > 0) HIPC(launch_copy_cols<double>(M.n, k, W, ld, Wi, P->L.ldk, P->s));
    const double s2 = M.residual(Wi, k);
    if (r) HIPC(hipMemcpyAsync(r, M.R->r, 8 * M.R->pl.nnz, hipMemcpyDeviceToDevice, P->s));
    if (deg) HIPC(hipMemcpyAsync(deg, M.deg, 8 * M.n, hipMemcpyDeviceToDevice, P->s));
    HIPC(hipStreamSynchronize(P->s));
    if (sumsq) *sumsq = s2;
  } catch (const BmgError &e) {
    return fail(e.st, e.msg);
  }
  return BMG_OK;
}

extern "C" bmg_status bmg_rke_solve(bmg_problem *P, double *W, int ld, const bmg_options *opt, int *k_out,
                                    bmg_result *res) {
  if (!opt || !W || !k_out) return fail(BMG_EINVAL, "bmg_rke_solve: null argument");
  if (ld < 8 || ld % 8) return fail(BMG_EINVAL, "bmg_rke_solve: ld must be a positive multiple of 8");
  if (!(opt->lambda > 0.0) || !(opt->alpha > 0.0) || opt->bm_epochs < 0 || opt->max_iter < 0 ||
      opt->ssi_max_iter < 1 || opt->k_init < 1)
    return fail(BMG_EINVAL, "bmg_rke_solve: bad options");
  bmg_status st = check_rke(P);
  if (st != BMG_OK) return st;
  try {
    RkeMethod M(P);
    int k = 0;
    st = M.solve(*opt, &k, res);
    REQUIRE(k <= ld, BMG_ENOMEM, "rank exceeds ld");
    if (k > 0) HIPC(launch_copy_cols<double>(M.n, k, M.last_W, P->L.ldk, W, ld, P->s));
    HIPC(hipStreamSynchronize(P->s));
    *k_out = k;
  } catch (const BmgError &e) {
    return fail(e.st, e.msg);
  }
  return st;
}

static bool step_rule_ok(const bmg_options *o) {
  if (o->step_rule == BMG_STEP_FIXED) return true;
  return o->step_rule == BMG_STEP_SPARSA && o->alpha_min > 0.0 && o->alpha_max >= o->alpha_min &&
         o->sparsa_beta > 0.0 && o->sparsa_beta < 1.0 && o->sparsa_delta > 0.0 &&
         o->sparsa_delta < 1.0 && std::isfinite(o->alpha_max);
}

extern "C" bmg_status bmg_prox_step(bmg_problem *P, double *W, double *H, int *k_inout, int ld,
                                    const bmg_options *opt, double *sigma, double *residual) {
  if (!k_inout || !opt) return fail(BMG_EINVAL, "bmg_prox_step: null argument");
  if (opt->lmsvd_p < 0 || opt->lmsvd_p > LMSVD_MAX_HIST || opt->ssi_max_iter < 1 ||
      !(opt->alpha > 0.0) || !step_rule_ok(opt))
    return fail(BMG_EINVAL, "bmg_prox_step: bad options");
  bmg_status st = check_factors(P, W, H, *k_inout, ld);
  if (st != BMG_OK) return st;
  try {
    Method<double> M(P);
    M.hist_p = opt->lmsvd_p;
    M.sparsa = opt->step_rule == BMG_STEP_SPARSA;
    M.sp_opt = *opt;
    if (M.sparsa) M.panel_on = false;
    Method<double>::State S;
    M.init_state(S);
    const int k = *k_inout;
    load_factors<double>(P, W, H, k, ld, S.W, S.H);
    // warm start from W~ alone: no previous prox output, no retained vector
    S.k = k; S.kc = 0; S.kp = 0;
    S.rank_cur = 0; S.rank_prev = 0; S.trunc_prev = 0;
    S.has_u = false;
    S.psi = opt->psi0;
    const double tau = opt->ssi_tol_floor;
    auto info = M.pg_step(S, true, opt->lambda, opt->alpha, tau, opt->ssi_max_iter, opt->seed, 0);
    REQUIRE(S.k <= ld, BMG_ENOMEM, "output rank exceeds ld");
    store_factors<double>(P, S.W, S.H, S.k, W, H, ld);
    HIPC(hipStreamSynchronize(P->s));
    *k_inout = S.k;
    if (sigma)
      for (int i = 0; i < S.k; ++i) sigma[i] = S.sigma[i];
    if (residual) *residual = info.residual;
  } catch (const BmgError &e) {
    return fail(e.st, e.msg);
  }
  return BMG_OK;
}

// ============================================================================ solve tasks
struct bmg::SolveTask {
  virtual ~SolveTask() {}
  virtual bool step() = 0;
  virtual bmg_status finish(double *W, double *H, int ld, int *k_out, bmg_result *res) = 0;
  bmg_problem *P = nullptr;
};

template <typename T, typename TG>
struct TypedTask : bmg::SolveTask {
  Method<T, TG> M;
  typename Method<T, TG>::State S;
  typename Method<T, TG>::Run r;
  TypedTask(bmg_problem *p, const bmg_options &o) : M(p) {
    P = p;
    M.solve_begin(o, S, r);
  }
  bool step() override { return M.solve_step(r); }
  bmg_status finish(double *W, double *H, int ld, int *k_out, bmg_result *res) override {
    const bmg_status st = M.solve_end(r, res);
    const int k = S.k;
    REQUIRE(k <= ld, BMG_ENOMEM, "rank exceeds ld");
    store_factors<T>(P, S.W, S.H, k, W, H, ld);
    HIPC(hipStreamSynchronize(P->s));
    if (k_out) *k_out = k;
    if (res) res->status = st;
    return st;
  }
};

bmg_status bmg::solve_task_create(bmg_problem *P, const bmg_options *opt, SolveTask **out) {
  if (!P || !opt || !out) return fail(BMG_EINVAL, "bmg_solve: null argument");
  *out = nullptr;
  if (opt->lambda <= 0.0 || opt->alpha <= 0.0 || opt->bm_epochs < 0 || opt->max_iter < 0 ||
      opt->ssi_max_iter < 1 || opt->k_init < 1 || opt->lmsvd_p < 0 ||
      opt->lmsvd_p > LMSVD_MAX_HIST || !step_rule_ok(opt) ||
      (opt->bm_solver != BMG_BM_PSD && opt->bm_solver != BMG_BM_POLYMF))
    return fail(BMG_EINVAL, "bmg_solve: bad options");
  P->reset_stats();
  P->timing = opt->timing != 0;
  try {
    if (P->prec == BMG_FP64) *out = new TypedTask<double, double>(P, *opt);
    else if (P->prec == BMG_FP32) *out = new TypedTask<float, float>(P, *opt);
    else *out = new TypedTask<float, bf16_t>(P, *opt);
  } catch (const BmgError &e) {
    P->timing = false;
    return fail(e.st, e.msg);
  }
  return BMG_OK;
}

bmg_status bmg::solve_task_step(SolveTask *t, int *done) {
  try {
    *done = t->step() ? 1 : 0;
  } catch (const BmgError &e) {
    t->P->timing = false;
    return fail(e.st, e.msg);
  }
  return BMG_OK;
}

bmg_status bmg::solve_task_finish(SolveTask *t, double *W, double *H, int ld, int *k_out,
                                  bmg_result *res) {
  try {
    const bmg_status st = t->finish(W, H, ld, k_out, res);
    t->P->timing = false;
    return st;
  } catch (const BmgError &e) {
    t->P->timing = false;
    if (res) res->status = e.st;
    return fail(e.st, e.msg);
  }
}

void bmg::solve_task_destroy(SolveTask *t) { delete t; }

extern "C" bmg_status bmg_solve(bmg_problem *P, double *W, double *H, int ld, const bmg_options *opt,
                                int *k_out, bmg_result *res) {
  if (!P || !opt || !W || !H) return fail(BMG_EINVAL, "bmg_solve: null argument");
  if (ld < 8 || ld % 8) return fail(BMG_EINVAL, "bmg_solve: ld must be a positive multiple of 8");
  SolveTask *t = nullptr;
  bmg_status st = solve_task_create(P, opt, &t);
  int done = 0;
  while (st == BMG_OK && !done) st = solve_task_step(t, &done);
  if (st == BMG_OK) st = solve_task_finish(t, W, H, ld, k_out, res);
  else if (res) res->status = st;
  solve_task_destroy(t);
  return st;
}

// ============================================================================ batcher API (serving)
namespace bmg {
PassBatcher *batcher_create() {
  PassBatcher *b = new PassBatcher();
  if (hipStreamCreateWithFlags(&b->bs, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return nullptr;
  }
  return b;
}
void batcher_destroy(PassBatcher *b) {
  if (!b) return;
  if (b->bs) {
    (void)hipStreamSynchronize(b->bs);
    (void)hipStreamDestroy(b->bs);
  }
  delete b;
}
void batcher_attach(bmg_problem *P, PassBatcher *b) {
  if (!P || !b) return;
  std::lock_guard<std::mutex> lk(b->mu);
  P->batcher = b;
  b->attached += 1;
}
void batcher_detach(bmg_problem *P) {
  if (!P || !P->batcher) return;
  PassBatcher *b = P->batcher;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    b->attached -= 1;
    P->batcher = nullptr;
  }
  b->cv.notify_all();   // a leader waiting for every attached problem re-checks
}
void batcher_stats(PassBatcher *b, long *launches, long *passes) {
  if (!b) return;
  std::lock_guard<std::mutex> lk(b->mu);
  if (launches) *launches = b->launches;
  if (passes) *passes = b->passes;
}
}  // namespace bmg
