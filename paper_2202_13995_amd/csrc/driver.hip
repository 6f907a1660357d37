// Host driver and C ABI of liblp.so.
//
// lu_factor runs the blocked right-looking LU of the paper's "Base
// Implementation" (section "High Performance Linpack", figure fig:lu_iteration)
// one block column of width nb at a time:
//   1. factor the column panel (diagonal block plus the "left" blocks below it)
//      with partial pivoting in one persistent launch (panel_fused.hip): the
//      workgroups split the panel's rows, exchange one candidate row per
//      column, and factor leaves of 16 or 32 columns held in registers;
//   2. apply the panel's row exchanges to every column outside the panel;
//   3. solve the "top" blocks with the panel's unit lower triangle;
//   4. update the "inner" blocks with one matrix multiplication.
// With look-ahead (figure fig:lu_execution_schedule_pcie: the communication
// phase of the next iteration overlaps the update phase), step 4 first updates
// only the next panel's columns, the next panel is factored on a second stream
// while the rest of the multiplication runs, and step 2/3 of the next
// iteration wait for both.  Steps 2/3 of the columns right of the next panel
// run on a third stream beside those of the next panel's own columns
// (binary64 / binary32), and step 2 left of the panel on a fourth.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"

namespace lp {


int num_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev >= 0 && dev < 64) {
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  if (dev >= 0 && dev < 64) cache[dev].store(cus, std::memory_order_relaxed);
  return cus;
}

namespace {

constexpr int kMaxN = 131072;
constexpr int kMaxNb = 1024;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Workspace layout of lu_factor (offsets in bytes).
// Row-exchange plans of consecutive steps live in a ring so that the exchanges
// left of the panel can run on their own stream, behind the main one.
constexpr int kPlanRing = 4;

struct FactorLayout {
  size_t barriers, n_barriers, slots, staging, keys0, keys1, plan_trail, plan_bytes, linv_trail,
      linv_left, linv_panel, pack_a, pack_b, total;
};

bool packs_operands(int prec) { return prec == LP_BF16 || prec == LP_FP16; }

FactorLayout factor_layout(int n, int nb, int prec) {
  FactorLayout L;
  size_t off = 0;
  L.barriers = off;
  L.n_barriers = (size_t)n + 64;
  off = align_up(off + 4 * L.n_barriers, 256);
  L.slots = off;
  off = align_up(off + leaf_slots_bytes(n, kLeafMax), 256);
  L.staging = off;
  off = align_up(off + panel_staging_bytes(kMaxNb), 256);
  L.keys0 = off;
  off = align_up(off + panel_keys_bytes(), 256);
  L.keys1 = off;
  off = align_up(off + panel_keys_bytes(), 256);
  L.plan_trail = off;  // a ring of kPlanRing plans (see factor_impl)
  L.plan_bytes = align_up(swap_plan_bytes(kMaxNb), 256);
  off += kPlanRing * L.plan_bytes;
  L.linv_trail = off;
  off = align_up(off + trsm_workspace_bytes(kMaxNb), 256);
  // block inverses of the no-pivot left-block solve (its own stream)
  L.linv_left = off;
  off = align_up(off + trsm_workspace_bytes(256), 256);
  // the block inverses inside a split panel (the panel's stream)
  L.linv_panel = off;
  off = align_up(off + trsm_workspace_bytes(kMaxNb / 2), 256);
  // bfloat16 / half: the packed operands of the trailing update (-L of the
  // step; U^T of a column range, placed at a 256-row offset per range)
  L.pack_a = L.pack_b = 0;
  if (packs_operands(prec)) {
    L.pack_a = off;
    off = align_up(off + gemm_lp_packed_bytes(n, nb), 256);
    L.pack_b = off;
    off = align_up(off + gemm_lp_packed_bytes(n + 1024, nb), 256);
  }
  L.total = off;
  return L;
}

bool valid_prec(int p) { return p == LP_FP64 || p == LP_FP32 || p == LP_BF16 || p == LP_FP16; }

template <typename T>
struct Factor {
  int m;  // rows
  T* A;
  long long lda;
  int32_t* ipiv;
  int32_t* info;
  char* slots;
  unsigned* barriers;
  int n_barriers;
  int next_barrier;
  void* staging;
  void* keys[2];  // per-launch key buffers, alternating; the first starts zeroed
  hipStream_t s;
  int max_w = 0;  // the widest panel launch of the factorization (key slots to clear)

  T* at(long long i, long long j) const { return A + i * lda + j; }

  // factor columns [j0, j0 + w) over rows [j0, m): one launch
  int panel(int j0, int w, int max_wgs = 0) {
    if (next_barrier >= n_barriers) return LP_ENOTSUP;
    const int idx = next_barrier++;
    unsigned* bar = barriers + idx;
    return launch_panel_fused<T>(m, j0, w, A, lda, ipiv, info, slots, bar, staging,
                                 keys[idx & 1], keys[(idx + 1) & 1], s, max_wgs, false, max_w);
  }

  // The same columns in two halves (partial pivoting, w >= 256): the left
  // half in one launch; its row exchanges, the "top" solve U12 = L11^-1 A12
  // and the update A22 -= L21 U12 applied to the right half; the right half
  // in a second launch; its row exchanges applied to the left half.  Inside
  // one launch the columns right of each leaf are read and written once per
  // leaf, so the panel moves about m w^2 / (2 leaf width) elements; the split
  // moves a quarter of that plus one rank-h product on the GEMM kernel.  The
  // pivots and the arithmetic of each element are those of partial pivoting;
  // only the grouping of the right half's updates changes.
  int panel_split(int j0, int w, int max_wgs, void* linv, int depth) {
    const int h = (w / 64) * 32;
    auto half = [&](int c, int ww) -> int {
      return (depth > 1 && ww >= 256) ? panel_split(c, ww, max_wgs, linv, depth - 1)
                                      : panel(c, ww, max_wgs);
    };
    int rc = half(j0, h);
    if (rc != LP_OK) return rc;
    if ((rc = launch_swap_fused<T>(A, lda, j0 + h, j0 + w, ipiv, j0, j0 + h, s)) != LP_OK)
      return rc;
    if ((rc = launch_trsm_lower_unit<T>(h, w - h, at(j0, j0), lda, at(j0, j0 + h), lda, linv,
                                        s)) != LP_OK)
      return rc;
    const int prec = sizeof(T) == 8 ? LP_FP64 : LP_FP32;
    if ((rc = launch_gemm_update(prec, m - j0 - h, w - h, h, at(j0 + h, j0), lda, at(j0, j0 + h),
                                 lda, at(j0 + h, j0 + h), lda, s, kGemmPanel)) != LP_OK)
      return rc;
    if ((rc = half(j0 + h, w - h)) != LP_OK) return rc;
    return launch_swap_fused<T>(A, lda, j0, j0 + h, ipiv, j0 + h, j0 + w, s);
  }

  // the same columns without pivoting, as the paper's LU and left kernels:
  // the w x w diagonal block in one workgroup (no pivot search; split as
  // below), then the blocks below it solved against its upper triangle,
  // L21 = A21 U11^-1
  int panel_nopiv(int j0, int w, void* linv_left, void* linv_diag, int depth) {
    int rc = diag_nopiv(j0, j0 + w, w, linv_diag, depth);
    if (rc != LP_OK || j0 + w >= m) return rc;
    return launch_trsm_right_upper<T>(m - j0 - w, w, at(j0, j0), lda, at(j0 + w, j0), lda,
                                      linv_left, s);
  }

  // LU without pivoting of columns [c, c + w) over rows [c, e) (e - c <= 1024,
  // one workgroup).  A block of 256 columns or more goes in two halves, split
  // `depth` times: the left half, then U12 = L11^-1 A12 and A22 -= L21 U12 on
  // the matrix cores, then the right half -- the same operations the one
  // launch applies leaf by leaf, a quarter of its in-kernel traffic.
  int diag_nopiv(int c, int e, int w, void* linv, int depth) {
    if (depth > 0 && w >= 256) {
      const int h = (w / 64) * 32;
      int rc = diag_nopiv(c, e, h, linv, depth - 1);
      if (rc != LP_OK) return rc;
      if ((rc = launch_trsm_lower_unit<T>(h, w - h, at(c, c), lda, at(c, c + h), lda, linv, s)) !=
          LP_OK)
        return rc;
      const int prec = sizeof(T) == 8 ? LP_FP64 : LP_FP32;
      if ((rc = launch_gemm_update(prec, e - c - h, w - h, h, at(c + h, c), lda, at(c, c + h), lda,
                                   at(c + h, c + h), lda, s, kGemmPanel)) != LP_OK)
        return rc;
      return diag_nopiv(c + h, e, w - h, linv, depth - 1);
    }
    if (next_barrier >= n_barriers) return LP_ENOTSUP;
    const int idx = next_barrier++;
    return launch_panel_fused<T>(e, c, w, A, lda, ipiv, info, slots, barriers + idx, staging,
                                 keys[idx & 1], keys[(idx + 1) & 1], s, 0, true);
  }
};

// Optional per-phase timing: HIP events bracket every launch group on the
// stream that runs it; read back after the call synchronizes.
struct Prof {
  bool on = false;
  struct Span {
    hipEvent_t a, b;
  };
  std::vector<Span> gemm, panel, swap, swapl, trsm;
  double gemm_flops = 0, gemm_bytes = 0, swap_bytes = 0, swapl_bytes = 0, trsm_flops = 0;

  int begin(std::vector<Span>& v, hipStream_t s) {
    if (!on) return LP_OK;
    Span sp;
    LP_HIP_TRY(hipEventCreate(&sp.a));
    LP_HIP_TRY(hipEventCreate(&sp.b));
    LP_HIP_TRY(hipEventRecord(sp.a, s));
    v.push_back(sp);
    return LP_OK;
  }
  int end(std::vector<Span>& v, hipStream_t s) {
    if (!on) return LP_OK;
    LP_HIP_TRY(hipEventRecord(v.back().b, s));
    return LP_OK;
  }
  static double total(std::vector<Span>& v) {
    double t = 0;
    for (auto& sp : v) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, sp.a, sp.b) == hipSuccess) t += ms;
    }
    return t;
  }
  void release() {
    for (auto* v : {&gemm, &panel, &swap, &swapl, &trsm})
      for (auto& sp : *v) {
        (void)hipEventDestroy(sp.a);
        (void)hipEventDestroy(sp.b);
      }
  }
};

// Look-ahead streams live for the process and are reused: destroying a stream
// waits for its work, which would make every factorization synchronous for
// the host.  A stream handed back may still hold work of the call that used it;
// a later call appends behind it (a false dependency, never a wrong order).
class StreamPool {
 public:
  hipError_t get(hipStream_t* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    {
      std::lock_guard<std::mutex> g(mu_);
      for (size_t i = 0; i < free_.size(); ++i)
        if (free_[i].dev == dev) {
          *out = free_[i].s;
          free_.erase(free_.begin() + (long)i);
          return hipSuccess;
        }
    }
    return hipStreamCreateWithFlags(out, hipStreamNonBlocking);
  }
  void put(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> g(mu_);
    free_.push_back({dev, s});
  }

 private:
  struct Entry {
    int dev;
    hipStream_t s;
  };
  std::mutex mu_;
  std::vector<Entry> free_;
};

StreamPool& stream_pool() {
  static StreamPool* pool = new StreamPool();  // never destroyed: streams outlive static teardown
  return *pool;
}

// Ordering events are reused the same way; one is handed out again only once
// it has completed, so no wait that names it can still be pending.
class EventPool {
 public:
  explicit EventPool(unsigned flags) : flags_(flags) {}
  hipError_t get(hipEvent_t* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    {
      std::lock_guard<std::mutex> g(mu_);
      for (size_t i = 0; i < free_.size(); ++i)
        if (free_[i].dev == dev && hipEventQuery(free_[i].e) == hipSuccess) {
          *out = free_[i].e;
          free_.erase(free_.begin() + (long)i);
          return hipSuccess;
        }
    }
    return hipEventCreateWithFlags(out, flags_);
  }
  void put(hipEvent_t ev) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> g(mu_);
    free_.push_back({dev, ev});
  }

 private:
  struct Entry {
    int dev;
    hipEvent_t e;
  };
  unsigned flags_;
  std::mutex mu_;
  std::vector<Entry> free_;
};

EventPool& event_pool() {
  static EventPool* pool = new EventPool(hipEventDisableTiming);
  return *pool;
}

EventPool& timing_event_pool() {
  static EventPool* pool = new EventPool(hipEventDefault);
  return *pool;
}

// RAII holder for the look-ahead streams and their events.
struct Lookahead {
  hipStream_t s2 = nullptr;  // the next panel
  hipStream_t s3 = nullptr;  // row exchanges left of the panel
  hipStream_t s4 = nullptr;  // exchanges and "top" solve right of the next panel
  // once panels are short: the panel on reserved compute units (sp), the rest
  // of the step (sr) and the left exchanges (sr2) on the others
  hipStream_t sp = nullptr, sr = nullptr, sr2 = nullptr;
  std::vector<hipEvent_t> ev;
  ~Lookahead() {
    for (auto e : ev) event_pool().put(e);
    for (hipStream_t x : {s2, s3, s4})
      if (x) stream_pool().put(x);
    for (hipStream_t x : {sp, sr, sr2})  // masked streams (optional mode): not pooled
      if (x) (void)hipStreamDestroy(x);
  }
  int event(hipEvent_t* out) {
    hipEvent_t e;
    LP_HIP_TRY(event_pool().get(&e));
    ev.push_back(e);
    *out = e;
    return LP_OK;
  }
};

// How one factorization schedules its work (lp_factor_opts).
struct FactorCfg {
  bool lookahead = true;
  int panel_cus = 0;
  int panel_rows = 0;
  bool pivot = true;  // false: the paper's elimination without row exchanges
  int split_rows = 0;  // panels of 256 columns or more and this many rows in two halves
};

// Streams restricted by compute-unit masks: the first `reserve` mask bits for
// the panel (the bits interleave over the XCDs, so every XCD gives
// reserve / 8 units) and the other bits for the rest of the step.  On failure
// the streams stay null and the factorization keeps the unmasked ones.
bool make_masked_streams(Lookahead& la, int ncu, int reserve) {
  std::vector<uint32_t> mp((ncu + 31) / 32, 0u), mr((ncu + 31) / 32, 0u);
  for (int b = 0; b < ncu; ++b) (b < reserve ? mp : mr)[b / 32] |= 1u << (b % 32);
  const uint32_t words = (uint32_t)mp.size();
  if (hipExtStreamCreateWithCUMask(&la.sp, words, mp.data()) == hipSuccess &&
      hipExtStreamCreateWithCUMask(&la.sr, words, mr.data()) == hipSuccess &&
      hipExtStreamCreateWithCUMask(&la.sr2, words, mr.data()) == hipSuccess)
    return true;
  (void)hipGetLastError();
  for (hipStream_t* x : {&la.sp, &la.sr, &la.sr2})
    if (*x) {
      (void)hipStreamDestroy(*x);
      *x = nullptr;
    }
  return false;
}

// Workgroups of a panel that runs beside the trailing update.  Binary64: 48
// of up to 1024 rows each (more when the rows need them) leave the other
// compute units to the update's FP64 MFMAs, which on one MI355X shortened the
// whole factorization (n = 32768 and 65536; 32, 48 and 64 within 4% of each
// other, 96 or more and one per 256 rows slower) although such a panel alone
// is slower than one spread over every compute unit.  Binary32 panels are the
// longer chain of the low-precision factorization for more of its steps: at
// most 128 workgroups (512 rows each above 32768 rows) measured best there
// (n = 65536: 0.94 against 1.00 s with one per 256 rows; 64 everywhere 1.50 s;
// with split panels at nb = 1024: 64 0.80 s, 96 0.75, 128 0.73, 160-256 0.74-0.76).
template <typename T>
int lookahead_panel_wgs(int rows) {
  return std::max(sizeof(T) == 8 ? 48 : 128, (int)cdiv(rows, kPanelRowsPerWg));
}

// Panels split in halves by default (rows in [min_rows, max_rows]).  Measured
// on one MI355X at n = 65536: in the bfloat16 / half factorizations the
// trailing update is bound by memory traffic and the panel is the longer
// chain, and the split gains at every size (nb = 512: 832 -> 800 ms; nb =
// 1024: 861 -> 736 ms with halves split again, 770 ms without).  Where the
// update is bound by the matrix cores, the extra launches on the panel's
// stream wait for compute units beside it and lengthen its chain while the
// update is long: binary64 3.17 s unsplit against 3.30 s splitting panels of
// 49152 rows or more and 3.48 s splitting all (n = 32768, nb = 256: 0.55
// against 0.64 s), binary32 2.54 against 2.64 s.  Short panels, which are
// the longer chain at the end of the factorization, gain: splitting those of
// at most 8192 rows took binary64 from 3.18 to 3.16 s (n = 32768: 0.534 to
// 0.531 s; at most 16384 rows: 0.537 s) and binary32 from 2.58 to 2.57 s.
struct SplitRule {
  int min_rows, max_rows;
};
SplitRule default_split(int prec) {
  return packs_operands(prec) ? SplitRule{1, INT_MAX} : SplitRule{1, 8192};
}
// halves of 256 columns or more are split again once (quarters of a 1024
// panel: 736 ms; a third level 737-749 ms)
constexpr int kSplitDepth = 2;
// the no-pivot diagonal block (512 x 512 in one workgroup at nb = 512) in two
// halves: the n = 65536 no-pivot solve 2.88 -> 2.84 s; halves split again:
// 3.00 s (more launches waiting for compute units beside the update)
constexpr int kNopivSplitDepth = 1;

template <typename T>
int factor_impl(int n, int nb, int prec, T* A, long long lda, int32_t* ipiv, int32_t* info,
                char* work, hipStream_t s, const FactorCfg& cfg, Prof& prof) {
  const FactorLayout L = factor_layout(n, nb, prec);
  int rc = launch_zero_words(info, 1, s);
  if (rc != LP_OK) return rc;
  if (n == 0) return LP_OK;
  if ((rc = launch_zero_words(work + L.barriers, L.n_barriers, s)) != LP_OK) return rc;
  if ((rc = launch_zero_words(work + L.keys0, panel_keys_bytes() / 4, s)) != LP_OK) return rc;
  if ((rc = launch_zero_words(work + L.slots, leaf_slots_bytes(n, kLeafMax) / 4, s)) != LP_OK)
    return rc;
  Factor<T> f{n, A, lda, ipiv, info, work + L.slots, (unsigned*)(work + L.barriers),
              (int)L.n_barriers, 0, work + L.staging, {work + L.keys0, work + L.keys1}, s};
  f.max_w = std::min(nb, n);  // a split panel's halves are narrower, its right half may be wider
  void* linv_trail = work + L.linv_trail;
  void* linv_left = work + L.linv_left;
  const bool piv = cfg.pivot;
  const SplitRule split = cfg.split_rows == 0  ? default_split(prec)
                          : cfg.split_rows > 0 ? SplitRule{cfg.split_rows, INT_MAX}
                                               : SplitRule{INT_MAX, 0};
  auto factor_panel = [&](int j0, int w, int max_wgs) -> int {
    if (!piv) return f.panel_nopiv(j0, w, linv_left, work + L.linv_panel, kNopivSplitDepth);
    if (w >= 256 && n - j0 >= split.min_rows && n - j0 <= split.max_rows)
      return f.panel_split(j0, w, max_wgs, work + L.linv_panel, kSplitDepth);
    return f.panel(j0, w, max_wgs);
  };
  char* plan_ring = work + L.plan_trail;
  void* plan_trail = plan_ring;  // the current step's plan
  const int npanels = (int)cdiv(n, nb);
  Lookahead la;
  if (cfg.lookahead && npanels > 1) {
    LP_HIP_TRY(stream_pool().get(&la.s2));
    LP_HIP_TRY(stream_pool().get(&la.s3));
    if (!packs_operands(prec)) LP_HIP_TRY(stream_pool().get(&la.s4));
  }
  // Optional reserved compute units for short panels.  While the trailing
  // update is long it hides the panel; once the panels are short they are the
  // longer chain, and on shared compute units their FP64 and LDS work queues
  // behind the update's.  With panel_cus set, the panel then runs on its own
  // units (at most one 1024-row workgroup each) and the update on the others.
  // Off by default: measured on one MI355X at n = 32768 and 65536 the panel
  // did not get faster on masked streams while the solve and exchanges on the
  // complement slowed down.
  const int ncu = num_cus();
  int reserve = cfg.panel_cus < 0 ? (ncu == 256 && n >= 8192 ? 32 : 0) : cfg.panel_cus;
  if (reserve < 8 || reserve % 8 != 0 || reserve >= ncu) reserve = 0;
  const int cap_rows = reserve * kPanelRowsPerWg;
  const int switch_rows =
      std::min(cfg.panel_rows > 0 ? cfg.panel_rows : std::min(cap_rows, 3 * (n / 4)), cap_rows);
  bool can_mask = la.s2 != nullptr && reserve > 0 && switch_rows > 0;
  hipStream_t ms = s;      // the step's swaps, solve and update
  hipStream_t ps = la.s2;  // the next panel
  hipStream_t ls = la.s3;  // exchanges left of the panel
  hipStream_t rs = la.s4;  // exchanges and "top" solve right of the next panel
                           // (binary64 / binary32 only, see below)
  int pwgs = 0;            // workgroup cap of panel launches (0: whole chip)
  // per ring slot: the left exchanges that read it; the main stream waits for
  // it before writing the slot again
  hipEvent_t left_done[kPlanRing] = {nullptr, nullptr, nullptr, nullptr};
  const double es = sizeof(T);
  int packed_step = -1;  // the step whose -L is in the packed buffer

  // Trailing steps of panel k over the column range [c0, c1) right of the
  // panel (and, if left, the columns left of the panel).  prepare: the row
  // exchanges and the "top" solve on stream st (with the block inverses
  // already in linv_trail when inv_ready); update: the multiplication on the
  // main stream; trailing: both on the main stream.
  auto prepare = [&](int j0, int w, int c0, int c1, bool left, hipStream_t st,
                     bool inv_ready) -> int {
    int r;
    if (piv) {
      if ((r = prof.begin(prof.swap, st)) != LP_OK) return r;
      if ((r = launch_swap_apply<T>(A, lda, c0, c1, 0, left ? j0 : 0, w, plan_trail, st)) !=
          LP_OK)
        return r;
      if ((r = prof.end(prof.swap, st)) != LP_OK) return r;
      prof.swap_bytes += 2.0 * es * 2.0 * w * ((c1 - c0) + (left ? j0 : 0));
    }
    if (c1 <= c0) return LP_OK;
    if ((r = prof.begin(prof.trsm, st)) != LP_OK) return r;
    if ((r = launch_trsm_lower_unit<T>(w, c1 - c0, f.at(j0, j0), lda, f.at(j0, c0), lda,
                                       linv_trail, st, inv_ready)) != LP_OK)
      return r;
    if ((r = prof.end(prof.trsm, st)) != LP_OK) return r;
    prof.trsm_flops += 1.0 * w * w * (c1 - c0);
    return LP_OK;
  };
  auto update = [&](int j0, int w, int c0, int c1) -> int {
    const int j1 = j0 + w;
    int r;
    if (c1 <= c0) return LP_OK;
    const int M = n - j1, N = c1 - c0;
    if (M <= 0) return LP_OK;
    if ((r = prof.begin(prof.gemm, ms)) != LP_OK) return r;
    if (L.pack_a != 0 && gemm_lp_packed_pays(prec, M, N, w)) {
      // -L packed once per step (both column ranges of the step run on this
      // stream, in order); U^T of this range at its own rows
      const size_t brow = (size_t)(c0 - j1 + 255) / 256 * 256;
      char* pb = work + L.pack_b + gemm_lp_packed_bytes((int)brow, w);
      r = launch_gemm_update_lp_packed(prec, M, N, w, (const float*)f.at(j1, j0), lda,
                                       (const float*)f.at(j0, c0), lda, (float*)f.at(j1, c0), lda,
                                       work + L.pack_a, pb, packed_step != j0, ms);
      if (r != LP_OK) return r;
      packed_step = j0;
    } else if ((r = launch_gemm_update(prec, M, N, w, f.at(j1, j0), lda, f.at(j0, c0), lda,
                                       f.at(j1, c0), lda, ms)) != LP_OK) {
      return r;
    }
    if ((r = prof.end(prof.gemm, ms)) != LP_OK) return r;
    prof.gemm_flops += 2.0 * M * N * w;
    prof.gemm_bytes += es * (2.0 * M * N + (double)M * w + (double)w * N);
    return LP_OK;
  };
  auto trailing = [&](int j0, int w, int c0, int c1, bool left) -> int {
    const int r = prepare(j0, w, c0, c1, left, ms, false);
    return r != LP_OK ? r : update(j0, w, c0, c1);
  };

  // panel 0 on the caller's stream
  if ((rc = prof.begin(prof.panel, s)) != LP_OK) return rc;
  if ((rc = factor_panel(0, std::min(nb, n), 0)) != LP_OK) return rc;
  if ((rc = prof.end(prof.panel, s)) != LP_OK) return rc;
  hipEvent_t panel_done = nullptr;  // event after the current panel (look-ahead stream)
  for (int k = 0; k < npanels; ++k) {
    const int j0 = k * nb;
    const int w = std::min(nb, n - j0);
    const int j1 = j0 + w;
    const bool more = k + 1 < npanels;
    const int w2 = more ? std::min(nb, n - j1) : 0;
    if (can_mask && more && n - j1 <= switch_rows) {
      // from this step on: everything after the work already queued, on the
      // masked streams
      can_mask = false;
      if (make_masked_streams(la, ncu, reserve)) {
        hipEvent_t e1, e2;
        if ((rc = la.event(&e1)) != LP_OK) return rc;
        LP_HIP_TRY(hipEventRecord(e1, ms));
        LP_HIP_TRY(hipStreamWaitEvent(la.sr, e1, 0));
        if ((rc = la.event(&e2)) != LP_OK) return rc;
        LP_HIP_TRY(hipEventRecord(e2, ls));
        LP_HIP_TRY(hipStreamWaitEvent(la.sr2, e2, 0));
        ms = la.sr;
        ps = la.sp;
        ls = la.sr2;
        rs = nullptr;  // the main stream waited for its last work
        pwgs = reserve;
      }
    }
    if (panel_done) LP_HIP_TRY(hipStreamWaitEvent(ms, panel_done, 0));
    const int slot = k % kPlanRing;
    plan_trail = plan_ring + (size_t)slot * L.plan_bytes;
    if (left_done[slot]) LP_HIP_TRY(hipStreamWaitEvent(ms, left_done[slot], 0));
    if (piv && (j0 > 0 || j1 < n)) {
      if ((rc = launch_swap_plan(ipiv, j0, j1, plan_trail, ms)) != LP_OK) return rc;
    }
    // With look-ahead, the exchanges and the "top" solve of the columns right
    // of the next panel run on their own stream, beside the same steps for
    // the next panel's own columns and their update on the main stream; both
    // ranges share one launch of L11's block inverses.  Not in the bfloat16 /
    // half factorizations (rs is not taken for them): there the panel chain
    // is the longer one for most steps, and the next panel's columns, which
    // are on that chain, slowed down beside the rest's exchanges and solve
    // (n = 65536, nb = 1024: 0.89 -> 1.19 ms from the end of a panel to the
    // start of the next).
    const bool side_rest = more && ps && rs && j1 + w2 < n;
    hipEvent_t rest_ready = nullptr;
    if (side_rest) {
      if ((rc = launch_diag_block_inverse<T>(w, f.at(j0, j0), lda, linv_trail, ms)) != LP_OK)
        return rc;
      hipEvent_t inv_ready;
      if ((rc = la.event(&inv_ready)) != LP_OK) return rc;
      LP_HIP_TRY(hipEventRecord(inv_ready, ms));
      LP_HIP_TRY(hipStreamWaitEvent(rs, inv_ready, 0));
      if ((rc = prepare(j0, w, j1 + w2, n, false, rs, true)) != LP_OK) return rc;
      if ((rc = la.event(&rest_ready)) != LP_OK) return rc;
      LP_HIP_TRY(hipEventRecord(rest_ready, rs));
    }
    if (piv && ls && j0 > 0) {
      // the exchanges left of the panel: nothing reads those columns before the
      // final join, so they run behind the main stream
      hipEvent_t plan_ready;
      if ((rc = la.event(&plan_ready)) != LP_OK) return rc;
      LP_HIP_TRY(hipEventRecord(plan_ready, ms));
      LP_HIP_TRY(hipStreamWaitEvent(ls, plan_ready, 0));
      if ((rc = prof.begin(prof.swapl, ls)) != LP_OK) return rc;
      if ((rc = launch_swap_apply<T>(A, lda, 0, j0, 0, 0, w, plan_trail, ls)) != LP_OK) return rc;
      if ((rc = prof.end(prof.swapl, ls)) != LP_OK) return rc;
      prof.swapl_bytes += 2.0 * es * 2.0 * w * j0;
      if ((rc = la.event(&left_done[slot])) != LP_OK) return rc;
      LP_HIP_TRY(hipEventRecord(left_done[slot], ls));
    }
    if (more && ps) {
      // the next panel's columns first, then factor it beside the rest
      if (side_rest) {
        if ((rc = prepare(j0, w, j1, j1 + w2, false, ms, true)) != LP_OK) return rc;
        if ((rc = update(j0, w, j1, j1 + w2)) != LP_OK) return rc;
      } else if ((rc = trailing(j0, w, j1, j1 + w2, false)) != LP_OK) {
        return rc;
      }
      hipEvent_t next_ready;
      if ((rc = la.event(&next_ready)) != LP_OK) return rc;
      LP_HIP_TRY(hipEventRecord(next_ready, ms));
      LP_HIP_TRY(hipStreamWaitEvent(ps, next_ready, 0));
      f.s = ps;
      if ((rc = prof.begin(prof.panel, ps)) != LP_OK) return rc;
      if ((rc = factor_panel(j1, w2, pwgs ? pwgs : lookahead_panel_wgs<T>(n - j1))) != LP_OK)
        return rc;
      if ((rc = prof.end(prof.panel, ps)) != LP_OK) return rc;
      f.s = s;
      if ((rc = la.event(&panel_done)) != LP_OK) return rc;
      LP_HIP_TRY(hipEventRecord(panel_done, ps));
      if (side_rest) {
        LP_HIP_TRY(hipStreamWaitEvent(ms, rest_ready, 0));
        if ((rc = update(j0, w, j1 + w2, n)) != LP_OK) return rc;
      } else if ((rc = trailing(j0, w, j1 + w2, n, ls == nullptr)) != LP_OK) {
        return rc;
      }
    } else {
      if ((rc = trailing(j0, w, j1, n, ls == nullptr)) != LP_OK) return rc;
      if (more) {
        f.s = ms;
        if ((rc = prof.begin(prof.panel, ms)) != LP_OK) return rc;
        if ((rc = factor_panel(j1, w2, 0)) != LP_OK) return rc;
        if ((rc = prof.end(prof.panel, ms)) != LP_OK) return rc;
        f.s = s;
      }
      panel_done = nullptr;
    }
  }
  // nothing may remain on the other streams past this point
  for (hipStream_t side : {la.s2, la.s3, la.s4, la.sp, la.sr, la.sr2}) {
    if (!side) continue;
    hipEvent_t joined;
    if ((rc = la.event(&joined)) != LP_OK) return rc;
    LP_HIP_TRY(hipEventRecord(joined, side));
    LP_HIP_TRY(hipStreamWaitEvent(s, joined, 0));
  }
  return LP_OK;
}

template <typename T>
int factor_entry(int n, int nb, int prec, T* A, long long lda, int32_t* ipiv, int32_t* info,
                 char* work, hipStream_t s, const FactorCfg& cfg, lp_factor_profile* out) {
  Prof prof;
  prof.on = out != nullptr;
  int rc = factor_impl<T>(n, nb, prec, A, lda, ipiv, info, work, s, cfg, prof);
  if (out != nullptr) {
    hipError_t e = hipStreamSynchronize(s);
    if (rc == LP_OK && e != hipSuccess) rc = LP_EHIP_BASE - (int)e;
    std::memset(out, 0, sizeof(*out));
    out->gemm_launches = (int)prof.gemm.size();
    out->gemm_ms = Prof::total(prof.gemm);
    out->gemm_flops = prof.gemm_flops;
    out->gemm_bytes = prof.gemm_bytes;
    out->panel_ms = Prof::total(prof.panel);
    out->panel_launches = (int)prof.panel.size();
    out->swap_ms = Prof::total(prof.swap);
    out->swap_bytes = prof.swap_bytes;
    out->swap_left_ms = Prof::total(prof.swapl);
    out->swap_left_bytes = prof.swapl_bytes;
    out->trsm_ms = Prof::total(prof.trsm);
    out->trsm_flops = prof.trsm_flops;
  }
  prof.release();
  return rc;
}

// Scratch of lu_factor_noalloc: a file-scope device array, so that callers
// that cannot allocate (code under graph capture, fixed serving loops) still
// get a factorization workspace.  Each device holds its own copy for the life
// of the process.  Host code never names the array directly (its host-side
// symbol is not a device address): the device address comes from
// hipGetSymbolAddress, once per device with that device current.
constexpr size_t kNoAllocScratchBytes = (size_t)8 << 20;
__device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

int scratch_address(void** out) {
  int dev = 0;
  LP_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return LP_ENOTSUP;
  std::lock_guard<std::mutex> g(scratch_mu);
  if (scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    LP_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return LP_OK;
}

}  // namespace

hipError_t acquire_timing_event(hipEvent_t* out) { return timing_event_pool().get(out); }
void release_timing_event(hipEvent_t e) { timing_event_pool().put(e); }

}  // namespace lp

using namespace lp;

extern "C" {

int lp_version(void) { return 100; }

const char* lp_strerror(int code) {
  if (code == LP_OK) return "success";
  if (code == LP_ENOSPC) return "workspace too small";
  if (code == LP_ENOTSUP) return "size or precision not supported by the kernels";
  if (code <= LP_EHIP_BASE) {
    const hipError_t e = (hipError_t)(LP_EHIP_BASE - code);
    return hipGetErrorString(e);
  }
  if (code < 0) return "illegal argument";
  return "unknown status";
}

size_t lu_workspace_bytes(int n, int nb, int prec) {
  if (n < 0 || n > kMaxN || nb < 1 || nb > kMaxNb || !valid_prec(prec)) return 0;
  return factor_layout(n, nb, prec).total;
}

int lu_factor_ex(int n, int nb, int prec, void* A, int lda, int32_t* ipiv, int32_t* info,
                 void* work, size_t work_bytes, const lp_factor_opts* opts,
                 lp_factor_profile* prof, void* stream) {
  if (n < 0) return -1;
  if (n > kMaxN) return LP_ENOTSUP;
  if (nb < 1 || nb > kMaxNb) return -2;
  if (!valid_prec(prec)) return -3;
  if (A == nullptr && n > 0) return -4;
  if (lda < std::max(1, n)) return -5;
  if (ipiv == nullptr && n > 0) return -6;
  if (info == nullptr) return -7;
  if (work == nullptr) return -8;
  if (work_bytes < lu_workspace_bytes(n, nb, prec)) return LP_ENOSPC;
  FactorCfg cfg;
  if (opts != nullptr) {
    cfg.lookahead = opts->lookahead != 0;
    cfg.panel_cus = opts->panel_cus;
    cfg.panel_rows = opts->panel_rows;
    cfg.pivot = opts->no_pivoting == 0;
    cfg.split_rows = opts->panel_split_rows;
  }
  hipStream_t s = (hipStream_t)stream;
  if (prec == LP_FP64)
    return factor_entry<double>(n, nb, prec, (double*)A, lda, ipiv, info, (char*)work, s, cfg,
                                prof);
  return factor_entry<float>(n, nb, prec, (float*)A, lda, ipiv, info, (char*)work, s, cfg, prof);
}

int lu_factor(int n, int nb, int prec, void* A, int lda, int32_t* ipiv, int32_t* info, void* work,
              size_t work_bytes, void* stream) {
  return lu_factor_ex(n, nb, prec, A, lda, ipiv, info, work, work_bytes, nullptr, nullptr, stream);
}

size_t lu_factor_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

int lu_factor_noalloc(int n, int nb, int prec, void* A, int lda, int32_t* ipiv, int32_t* info,
                      void* stream) {
  if (n < 0) return -1;
  if (n > kMaxN) return LP_ENOTSUP;
  if (nb < 1 || nb > kMaxNb) return -2;
  if (!valid_prec(prec)) return -3;
  if (prec != LP_FP64 && prec != LP_FP32) return LP_ENOTSUP;  // packed operands need more
  if (A == nullptr && n > 0) return -4;
  if (lda < std::max(1, n)) return -5;
  if (ipiv == nullptr && n > 0) return -6;
  if (info == nullptr) return -7;
  if (lu_workspace_bytes(n, nb, prec) > kNoAllocScratchBytes) return LP_ENOSPC;
  void* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc != LP_OK) return rc;
  FactorCfg cfg;
  cfg.lookahead = false;  // one stream: no internal streams or events to create
  hipStream_t s = (hipStream_t)stream;
  if (prec == LP_FP64)
    return factor_entry<double>(n, nb, prec, (double*)A, lda, ipiv, info, (char*)ws, s, cfg,
                                nullptr);
  return factor_entry<float>(n, nb, prec, (float*)A, lda, ipiv, info, (char*)ws, s, cfg, nullptr);
}

int lu_factor_nopiv(int n, int nb, int prec, void* A, int lda, int32_t* ipiv, int32_t* info,
                    void* work, size_t work_bytes, void* stream) {
  lp_factor_opts o;
  o.lookahead = 1;
  o.panel_cus = 0;
  o.panel_rows = 0;
  o.no_pivoting = 1;
  o.panel_split_rows = 0;
  return lu_factor_ex(n, nb, prec, A, lda, ipiv, info, work, work_bytes, &o, nullptr, stream);
}

int lu_solve(int n, int storage, const void* LU, int lda, const int32_t* ipiv,
             const int32_t* info, void* B, int ldb, int nrhs, int32_t* solve_status,
             void* stream) {
  if (n < 0) return -1;
  if (storage != LP_FP64 && storage != LP_FP32) return -2;
  if (LU == nullptr && n > 0) return -3;
  if (lda < std::max(1, n)) return -4;
  if (ipiv == nullptr && n > 0) return -5;
  if (B == nullptr && n > 0 && nrhs > 0) return -7;
  if (nrhs < 0) return -9;
  if (ldb < std::max(1, nrhs)) return -8;
  hipStream_t s = (hipStream_t)stream;
  if (storage == LP_FP64)
    return launch_lu_solve<double>(n, (const double*)LU, lda, ipiv, info, (double*)B, ldb, nrhs,
                                   solve_status, s);
  return launch_lu_solve<float>(n, (const float*)LU, lda, ipiv, info, (float*)B, ldb, nrhs,
                                solve_status, s);
}

size_t lu_solve_workspace_bytes(int n, int storage, int nrhs) {
  if (n < 0 || nrhs < 0 || (storage != LP_FP64 && storage != LP_FP32)) return 0;
  return lu_solve_workspace_bytes_t(n, storage == LP_FP64 ? 8 : 4);
}

int lu_solve_ex(int n, int storage, const void* LU, int lda, const int32_t* ipiv,
                const int32_t* info, void* B, int ldb, int nrhs, int32_t* solve_status,
                void* work, size_t work_bytes, void* stream) {
  if (n < 0) return -1;
  if (storage != LP_FP64 && storage != LP_FP32) return -2;
  if (LU == nullptr && n > 0) return -3;
  if (lda < std::max(1, n)) return -4;
  if (ipiv == nullptr && n > 0) return -5;
  if (B == nullptr && n > 0 && nrhs > 0) return -7;
  if (nrhs < 0) return -9;
  if (ldb < std::max(1, nrhs)) return -8;
  if (work == nullptr) return -11;
  if (work_bytes < lu_solve_workspace_bytes(n, storage, nrhs)) return LP_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  if (storage == LP_FP64)
    return launch_lu_solve_ws<double, double>(n, (const double*)LU, lda, ipiv, info, (double*)B,
                                              ldb, nrhs, solve_status, work, s);
  return launch_lu_solve_ws<float, float>(n, (const float*)LU, lda, ipiv, info, (float*)B, ldb,
                                          nrhs, solve_status, work, s);
}

int residual_check(int n, const double* A, int lda, const double* X, int ldx, const double* B,
                   int ldb, int nrhs, double* out, void* stream) {
  if (n < 0) return -1;
  if (A == nullptr && n > 0) return -2;
  if (lda < std::max(1, n)) return -3;
  if (X == nullptr && n > 0) return -4;
  if (ldx < std::max(1, nrhs)) return -5;
  if (B == nullptr && n > 0) return -6;
  if (ldb < std::max(1, nrhs)) return -7;
  if (nrhs < 0) return -8;
  if (out == nullptr && nrhs > 0) return -9;
  return launch_residual(n, A, lda, X, ldx, B, ldb, nrhs, out, (hipStream_t)stream, nullptr, 0);
}

int lp_panel_factor(int m, int w, int prec, void* A, int lda, int32_t* ipiv, int32_t* info,
                    void* work, size_t work_bytes, int max_wgs, void* stream) {
  if (m < 0 || m > kMaxN) return -1;
  if (w < 0 || w > m || w > kMaxNb) return -2;
  if (!valid_prec(prec)) return -3;
  if (A == nullptr && m > 0) return -4;
  if (lda < std::max(1, w)) return -5;
  if (ipiv == nullptr && w > 0) return -6;
  if (info == nullptr) return -7;
  if (work == nullptr) return -8;
  if (work_bytes < lu_workspace_bytes(m, std::max(1, w), prec)) return LP_ENOSPC;
  if (max_wgs < 0) return -10;
  hipStream_t s = (hipStream_t)stream;
  const FactorLayout L = factor_layout(m, std::max(1, w), prec);
  int rc = launch_zero_words(info, 1, s);
  if (rc != LP_OK || w == 0) return rc;
  if ((rc = launch_zero_words((char*)work + L.barriers, L.n_barriers, s)) != LP_OK) return rc;
  char* wk = (char*)work;
  if ((rc = launch_zero_words(wk + L.keys0, panel_keys_bytes() / 4, s)) != LP_OK) return rc;
  if ((rc = launch_zero_words(wk + L.slots, leaf_slots_bytes(m, kLeafMax) / 4, s)) != LP_OK)
    return rc;
  if (prec == LP_FP64) {
    Factor<double> f{m, (double*)A, lda, ipiv, info, wk + L.slots,
                     (unsigned*)(wk + L.barriers), (int)L.n_barriers, 0, wk + L.staging,
                     {wk + L.keys0, wk + L.keys1}, s};
    return f.panel(0, w, max_wgs);
  }
  Factor<float> f{m, (float*)A, lda, ipiv, info, wk + L.slots,
                  (unsigned*)(wk + L.barriers), (int)L.n_barriers, 0, wk + L.staging,
                  {wk + L.keys0, wk + L.keys1}, s};
  return f.panel(0, w, max_wgs);
}

size_t lp_laswp_workspace_bytes(int nswaps) {
  if (nswaps < 0 || nswaps > kMaxNb) return 0;
  return swap_plan_bytes(nswaps);
}

int lp_laswp(int prec, void* A, int lda, int c0, int c1, int k1, int k2, const int32_t* ipiv,
             void* work, size_t work_bytes, void* stream) {
  if (!valid_prec(prec)) return -1;
  if (lda < 1) return -3;
  if (c0 < 0 || c0 > lda) return -4;
  if (c1 < c0 || c1 > lda) return -5;
  if (k1 < 0) return -6;
  if (k2 < k1 || k2 - k1 > kMaxNb) return -7;
  if (ipiv == nullptr && k2 > k1) return -8;
  if (A == nullptr && k2 > k1 && c1 > c0) return -2;
  if (work == nullptr) return -9;
  if (work_bytes < lp_laswp_workspace_bytes(k2 - k1)) return LP_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  if (k2 == k1 || c1 == c0) return LP_OK;
  int rc = launch_swap_plan(ipiv, k1, k2, work, s);
  if (rc != LP_OK) return rc;
  if (prec == LP_FP64)
    return launch_swap_apply<double>((double*)A, lda, c0, c1, c1, c1, k2 - k1, work, s);
  return launch_swap_apply<float>((float*)A, lda, c0, c1, c1, c1, k2 - k1, work, s);
}

size_t lp_trsm_workspace_bytes(int m) {
  if (m < 0) return 0;
  return trsm_workspace_bytes(std::max(m, 1));  // the inverses of all diagonal blocks
}

int lp_trsm_lower_unit(int prec, int m, int ncols, const void* L, int ldl, void* B, int ldb,
                       void* work, size_t work_bytes, void* stream) {
  if (!valid_prec(prec)) return -1;
  if (m < 0) return -2;
  if (ncols < 0) return -3;
  if (L == nullptr && m > 0) return -4;
  if (ldl < std::max(1, m)) return -5;
  if (B == nullptr && m > 0 && ncols > 0) return -6;
  if (ldb < std::max(1, ncols)) return -7;
  if (work == nullptr) return -8;
  if (work_bytes < lp_trsm_workspace_bytes(m)) return LP_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  if (prec == LP_FP64)
    return launch_trsm_lower_unit<double>(m, ncols, (const double*)L, ldl, (double*)B, ldb, work,
                                          s);
  return launch_trsm_lower_unit<float>(m, ncols, (const float*)L, ldl, (float*)B, ldb, work, s);
}

size_t lp_trsm_right_workspace_bytes(int w) {
  if (w < 0) return 0;
  return trsm_workspace_bytes(std::min(std::max(w, 1), 128));
}

int lp_trsm_right_upper(int prec, int m, int w, const void* U, int ldu, void* B, int ldb,
                        void* work, size_t work_bytes, void* stream) {
  if (!valid_prec(prec)) return -1;
  if (m < 0) return -2;
  if (w < 0 || w > kMaxNb) return -3;
  if (U == nullptr && w > 0) return -4;
  if (ldu < std::max(1, w)) return -5;
  if (B == nullptr && m > 0 && w > 0) return -6;
  if (ldb < std::max(1, w)) return -7;
  if (work == nullptr) return -8;
  if (work_bytes < lp_trsm_right_workspace_bytes(w)) return LP_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  if (prec == LP_FP64)
    return launch_trsm_right_upper<double>(m, w, (const double*)U, ldu, (double*)B, ldb, work, s);
  return launch_trsm_right_upper<float>(m, w, (const float*)U, ldu, (float*)B, ldb, work, s);
}

int lp_gemm_update(int prec, int M, int N, int K, const void* A, int lda, const void* B, int ldb,
                   void* C, int ldc, void* stream) {
  if (!valid_prec(prec)) return -1;
  if (M < 0) return -2;
  if (N < 0) return -3;
  if (K < 0) return -4;
  if (A == nullptr && M > 0 && K > 0) return -5;
  if (lda < std::max(1, K)) return -6;
  if (B == nullptr && K > 0 && N > 0) return -7;
  if (ldb < std::max(1, N)) return -8;
  if (C == nullptr && M > 0 && N > 0) return -9;
  if (ldc < std::max(1, N)) return -10;
  return launch_gemm_update(prec, M, N, K, A, lda, B, ldb, C, ldc, (hipStream_t)stream);
}

size_t lp_gemm_packed_workspace_bytes(int M, int N, int K) {
  if (M < 0 || N < 0 || K < 0 || K > 1024) return 0;
  const size_t a = gemm_lp_packed_bytes(std::max(M, 1), std::max(K, 1));
  return align_up(a, 256) + gemm_lp_packed_bytes(std::max(N, 1), std::max(K, 1));
}

int lp_gemm_update_packed(int prec, int M, int N, int K, const void* A, int lda, const void* B,
                          int ldb, void* C, int ldc, void* work, size_t work_bytes, void* stream) {
  if (!packs_operands(prec)) return -1;
  if (M < 0) return -2;
  if (N < 0) return -3;
  if (K < 0 || K > 1024) return -4;
  if (A == nullptr && M > 0 && K > 0) return -5;
  if (lda < std::max(1, K)) return -6;
  if (B == nullptr && K > 0 && N > 0) return -7;
  if (ldb < std::max(1, N)) return -8;
  if (C == nullptr && M > 0 && N > 0) return -9;
  if (ldc < std::max(1, N)) return -10;
  if (work == nullptr) return -11;
  if (work_bytes < lp_gemm_packed_workspace_bytes(M, N, K)) return LP_ENOSPC;
  if (M == 0 || N == 0 || K == 0) return LP_OK;
  char* w = (char*)work;
  return launch_gemm_update_lp_packed(
      prec, M, N, K, (const float*)A, lda, (const float*)B, ldb, (float*)C, ldc, w,
      w + align_up(gemm_lp_packed_bytes(M, K), 256), true, (hipStream_t)stream);
}

int lp_ptrans(int prec, int n, const void* A, int lda, const void* B, int ldb, void* C, int ldc,
              void* stream) {
  if (prec != LP_FP64 && prec != LP_FP32) return -1;
  if (n < 0) return -2;
  if (A == nullptr && n > 0) return -3;
  if (lda < std::max(1, n)) return -4;
  if (B == nullptr && n > 0) return -5;
  if (ldb < std::max(1, n)) return -6;
  if (C == nullptr && n > 0) return -7;
  if (ldc < std::max(1, n)) return -8;
  return launch_ptrans(prec, n, A, lda, B, ldb, C, ldc, (hipStream_t)stream);
}

int lp_convert(int to_f32, int rows, int cols, const void* src, int lds, void* dst, int ldd,
               void* stream) {
  if (rows < 0) return -2;
  if (cols < 0) return -3;
  if (src == nullptr && rows > 0 && cols > 0) return -4;
  if (lds < std::max(1, cols)) return -5;
  if (dst == nullptr && rows > 0 && cols > 0) return -6;
  if (ldd < std::max(1, cols)) return -7;
  return launch_convert(to_f32, rows, cols, src, lds, dst, ldd, (hipStream_t)stream);
}

}  // extern "C"
