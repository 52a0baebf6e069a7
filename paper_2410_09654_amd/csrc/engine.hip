// Host orchestration and C ABI of the Pauli-string engine (see include/pauli.h).
//
// Every operation is one or more "engine calls": records from a commutator
// pair loop and/or from operator terms are binned by the leading bits of
// their mixed key, merged per bucket in LDS (summing each string's
// contributions in canonical order), filtered, reduced to the top-M by an
// exact radix select and compacted into the output.  The engine carves all
// of its scratch from the caller's workspace; intermediate operators of a
// Runge-Kutta step live at the top end of the same workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pauli.h"
#include "kernels.hpp"
#include "select.hpp"
#include "mlp.hpp"

using namespace pauli;

namespace {

thread_local std::string g_last_error;
thread_local pauli_stats g_stats;
thread_local pauli_totals g_totals;

// ---------------------------------------------------------------------------
// Optional kernel timing
// ---------------------------------------------------------------------------
struct Prof {
  std::mutex mu;
  bool on = false;
  std::set<std::string> only;  // kernel names to time; empty: every kernel
  struct Pending {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<long, double>> acc;

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void resolve() {  // call after the stream is synchronised
    std::lock_guard<std::mutex> g(mu);
    for (auto& p : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        auto& e = acc[p.name];
        e.first += 1;
        e.second += ms;
      }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
};
Prof g_prof;

struct ProfScope {
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(const char* n, hipStream_t st) : name(n), s(st) {
    if (!g_prof.on) return;
    std::lock_guard<std::mutex> g(g_prof.mu);
    if (!g_prof.only.empty() && !g_prof.only.count(n)) return;
    a = g_prof.get();
    b = g_prof.get();
    if (a) (void)hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (!a || !b) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> g(g_prof.mu);
    g_prof.pending.push_back({name, a, b});
  }
};

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      g_last_error = std::string(#expr) + ": " + hipGetErrorString(e_);           \
      return PAULI_EHIP;                                                           \
    }                                                                              \
  } while (0)

#define LAUNCH(name, kern, grid, block, ...)                                       \
  do {                                                                             \
    ProfScope ps_(name, stream);                                                   \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, stream, __VA_ARGS__);     \
    HIP_TRY(hipGetLastError());                                                    \
  } while (0)

#define TRY(expr)                    \
  do {                               \
    int rc_ = (expr);                \
    if (rc_ != PAULI_OK) return rc_; \
  } while (0)

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
inline int words_of(int n_qubits) { return (n_qubits + 63) / 64; }

// pinned host copy of the control block (one per thread)
thread_local Ctl* t_hctl = nullptr;
thread_local hipEvent_t t_ctl_event = nullptr, t_scan_event = nullptr;
thread_local hipStream_t t_side_stream = nullptr;  // on device t_side_dev
thread_local int t_side_dev = -1;
int host_ctl(Ctl** out) {
  if (!t_hctl) HIP_TRY(hipHostMalloc((void**)&t_hctl, sizeof(Ctl), hipHostMallocDefault));
  *out = t_hctl;
  return PAULI_OK;
}

// ---------------------------------------------------------------------------
// Workspace arena: engine scratch grows from the bottom (reset per engine
// call), operators that outlive an engine call are taken from the top.
// ---------------------------------------------------------------------------
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t bottom = 0;  // next free byte from the bottom
  size_t top = 0;     // bytes used at the top end
  size_t need = 0;    // largest bottom + top requested so far
  bool short_ = false;

  bool dry = false;    // size only (pauli_workspace_query): no memory behind it

  void* take(size_t bytes) {
    bottom = align256(bottom);
    const size_t at = bottom;
    bottom += align256(bytes);
    if (bottom + top > need) need = bottom + top;
    if (dry) return nullptr;
    if (bottom + top > cap) {
      short_ = true;
      return nullptr;
    }
    return base + at;
  }
  void* take_top(size_t bytes) {
    top += align256(bytes);
    if (bottom + top > need) need = bottom + top;
    if (dry) return nullptr;
    if (bottom + top > cap) {
      short_ = true;
      return nullptr;
    }
    return base + (cap - top);
  }
};

struct OpV {
  int W = 1;
  int f32 = 0;
  int canon = 0;  // written by the engine: canonical order known
  int64_t n = 0;
  int64_t cap = 0;
  const uint64_t* x = nullptr;
  const uint64_t* z = nullptr;
  const void* c = nullptr;
};

OpV view(const pauli_op* o) {
  OpV v;
  v.W = words_of(o->n_qubits);
  v.f32 = o->dtype == PAULI_C64K;
  v.n = o->size;
  v.cap = o->capacity;
  v.x = o->x;
  v.z = o->z;
  v.c = o->coef;
  return v;
}

int check_op(const pauli_op* o, bool output) {
  if (!o) return PAULI_EINVAL;
  if (o->n_qubits < 1 || o->n_qubits > 128) return PAULI_EINVAL;
  if (o->dtype != PAULI_C128 && o->dtype != PAULI_C64K) return PAULI_EINVAL;
  if (o->capacity < 0 || (!output && (o->size < 0 || o->size > o->capacity))) return PAULI_EINVAL;
  if (o->capacity > 0 && (!o->x || !o->z || !o->coef)) return PAULI_EINVAL;
  return PAULI_OK;
}

struct GroupSpec {
  int kind = G_TERM;
  double2 alpha = make_double2(1.0, 0.0);
  bool divide = false;  // the group's values are divided by alpha.x instead
};

struct OutSpec {
  pauli_op* user = nullptr;  // write into the caller's operator
  bool to_arena = false;     // or allocate at the top of the workspace
  OpV arena_op;              // filled when to_arena
  int f32 = 0;
};

struct Call {
  int W = 1;
  bool f32rec = false;  // FP32 record values (precision split)
  bool has_comm = false;
  bool product = false;  // A B instead of [A, B] (H = A, O = B)
  int ts = 0;  // > 0: translation-symmetric operators on ts periodic sites (Alg. 2)
  OpV H, O;
  int comm_group = 0;
  int n_terms = 0;
  OpV T[MAX_TERMS];
  int tgroup[MAX_TERMS] = {0};
  int tlist[MAX_TERMS] = {0};
  int n_groups = 0;
  GroupSpec groups[MAX_GROUPS];
  int mode = M_PLAIN;
  bool round32 = false;
  const pauli_trunc* trunc = nullptr;
  OutSpec out;
  // Lanczos
  double b_prev = 0.0;
  double* b_out = nullptr;
};

int alpha_kind(double2 a) {
  if (a.x == 1.0 && a.y == 0.0) return A_ONE;
  if (a.x == 0.0 && a.y == 1.0) return A_I;
  return A_GENERAL;
}

// ---------------------------------------------------------------------------
// Planning and scratch layout of one engine call, shared by the engine and
// pauli_workspace_query (which lays the same buffers out on an empty arena).
// ---------------------------------------------------------------------------
// at most 1024 commutator rows (one tile of EMIT_THREADS O strings each up
// to |O| = 2^20: more, shorter rows scatter faster, since twice as many
// workgroups fit a CU as there are CUs) and 128 rows of operator terms
constexpr int64_t COMM_ROWS_MAX = 1024, TERM_ROWS_MAX = (1 << 17) / EMIT_THREADS;
static_assert(COMM_ROWS_MAX + TERM_ROWS_MAX <= SC_ROWS_MAX, "k_scan_cols covers every count row");
constexpr int MAX_PASS_BITS = 12;
constexpr int DIRECT_MAX_F = 22;  // at most 2^22 buckets in a direct merge
constexpr int PART_NBL = 12;  // at most 2^12 partitions (MAX_PASS_BITS)
// blocks binning one partition: 1024 (one per CU, LDS-bound, so four
// rounds) write shorter per-(block, bin) runs and beat 256 and 512
constexpr int SPLIT_ROWS = 1024;
static_assert(SPLIT_ROWS <= SC_ROWS_MAX, "k_scan_cols covers every split row");

inline void plan_rows(bool comm, int64_t nO, int64_t nterm_rec, int* comm_rows, int* term_rows) {
  *comm_rows = comm ? (int)std::min<int64_t>((nO + EMIT_THREADS - 1) / EMIT_THREADS, COMM_ROWS_MAX) : 0;
  *term_rows = nterm_rec > 0
                   ? (int)std::min<int64_t>((nterm_rec + EMIT_THREADS - 1) / EMIT_THREADS, TERM_ROWS_MAX)
                   : 0;
}

// Hash passes from the largest bin of the NBINS_LOG-bin count: one pass when
// every bin fits a merge bucket; otherwise NBINS_LOG_MP bins per pass, whose
// largest holds about half as many, and one more pass bit per halving.
template <int W>
int plan_pass_bits(unsigned long long mx, int* nbl) {
  int pass_bits = 0;
  *nbl = NBINS_LOG;
  if (mx > (unsigned long long)merge_cap<W>()) {
    *nbl = NBINS_LOG_MP;
    mx = (mx + 1) / 2;
    while (mx > (unsigned long long)(merge_cap<W>() * 3 / 4) && pass_bits < 10) {
      pass_bits++;
      mx = (mx + 1) / 2;
    }
  }
  return pass_bits;
}

// scratch taken before the count pass
template <int W>
struct Bufs1 {
  Ctl* dctl = nullptr;
  uint64_t* Hk = nullptr;
  uint32_t* Hidx = nullptr;
  uint32_t* hstart = nullptr;
  int* hspan = nullptr;
  Key<W>* keep_mk = nullptr;
  uint32_t *counts = nullptr, *bin_total = nullptr, *bin_base = nullptr, *hist0 = nullptr;
  uint32_t* histL[2] = {nullptr, nullptr};
  uint32_t *hsum = nullptr, *h0sum = nullptr;
  unsigned long long* psum = nullptr;
  uint32_t* defer = nullptr;  // buckets left to the full-size merge (per pass)
};
template <int W>
void take_bufs1(Arena& ar, bool comm, int64_t nH, int64_t n_keep, int rows, Bufs1<W>& b) {
  const size_t KB = sizeof(Key<W>);
  b.dctl = (Ctl*)ar.take(sizeof(Ctl));
  b.Hk = comm ? (uint64_t*)ar.take((size_t)nH * KB) : nullptr;
  b.Hidx = comm ? (uint32_t*)ar.take((size_t)nH * 4) : nullptr;
  b.hstart = comm ? (uint32_t*)ar.take((size_t)(64 * W + 2) * 4) : nullptr;
  b.hspan = comm ? (int*)ar.take(4) : nullptr;
  b.keep_mk = n_keep ? (Key<W>*)ar.take((size_t)n_keep * KB) : nullptr;
  // rows of the emission, or of the partition binning (256 blocks)
  b.counts = (uint32_t*)ar.take((size_t)std::max(rows, 256) * NBINS_MP * 4);
  b.bin_total = (uint32_t*)ar.take(NBINS_MP * 4);
  b.bin_base = (uint32_t*)ar.take((NBINS_MP + 1) * 4);
  b.hist0 = (uint32_t*)ar.take((size_t)HREP * SEL0_BINS * 4);
  b.histL[0] = (uint32_t*)ar.take((size_t)HREP * SEL_BINS * 4);
  b.histL[1] = (uint32_t*)ar.take((size_t)HREP * SEL_BINS * 4);
  b.hsum = (uint32_t*)ar.take(SEL_BINS * 4);
  b.h0sum = (uint32_t*)ar.take(SEL0_BINS * 4);
  b.psum = (unsigned long long*)ar.take(PLAN_PARTS * 4 * 8);
  b.defer = (uint32_t*)ar.take(NBINS_MP * 4);
}

// scratch taken after the count pass: records (and their partitions),
// merged strings, per-bucket tables, select candidate lists
struct Bufs2 {
  void* recs = nullptr;
  uint32_t* rsrc_wide = nullptr;
  void* precs = nullptr;
  uint32_t *ptop = nullptr, *psrc = nullptr, *pbase = nullptr, *scounts = nullptr;
  void* uk = nullptr;
  double2* uc = nullptr;
  uint32_t *b_ubase = nullptr, *b_slots = nullptr, *b_surv = nullptr, *b_keep = nullptr;
  uint32_t *b_unique = nullptr, *b_abv = nullptr, *b_bcnt = nullptr, *b_obase = nullptr;
  double2* norm_part = nullptr;
  uint32_t* cand[3] = {nullptr, nullptr, nullptr};
  uint32_t* ccnt[3] = {nullptr, nullptr, nullptr};
};
template <int W, bool F32>
void take_bufs2(Arena& ar, size_t ptot, bool wide, bool partitioned, uint32_t max_buckets,
                bool want_select, Bufs2& b, bool records = true) {
  const size_t KB = sizeof(Key<W>), RB = sizeof(Rec<W, F32>);
  b.recs = records ? ar.take(ptot * RB) : nullptr;
  b.rsrc_wide = wide ? (uint32_t*)ar.take(ptot * 4) : nullptr;
  // several passes: every record is emitted once into 2^pass_bits partitions
  // (the top 32 bits of its order key aside, and its source id when wide);
  // each pass bins one partition
  b.precs = partitioned ? ar.take(ptot * RB) : nullptr;
  b.ptop = partitioned ? (uint32_t*)ar.take(ptot * 4) : nullptr;
  b.psrc = partitioned && wide ? (uint32_t*)ar.take(ptot * 4) : nullptr;
  b.pbase = partitioned ? (uint32_t*)ar.take(((1u << PART_NBL) + 1) * 4) : nullptr;
  b.scounts = partitioned ? (uint32_t*)ar.take((size_t)SPLIT_ROWS * NBINS_MP * 4) : nullptr;
  b.uk = ar.take(ptot * KB);
  b.uc = (double2*)ar.take(ptot * sizeof(double2));
  uint32_t** tabs[8] = {&b.b_ubase, &b.b_slots, &b.b_surv,  &b.b_keep,
                        &b.b_unique, &b.b_abv,  &b.b_bcnt, &b.b_obase};
  for (auto t : tabs) *t = (uint32_t*)ar.take((size_t)max_buckets * 4);
  b.norm_part = (double2*)ar.take((size_t)max_buckets * sizeof(double2));
  if (want_select)
    for (int k = 0; k < 3; k++) {
      b.cand[k] = (uint32_t*)ar.take(ptot * 4);
      b.ccnt[k] = (uint32_t*)ar.take((size_t)max_buckets * 4);
    }
}

struct Engine {
  Arena* ar;
  hipStream_t stream;
  Ctl* dctl = nullptr;
  Ctl* hctl = nullptr;
  // the count's copy to the host beside the scatter (pinned control block only):
  // recorded after the scan on the call's stream, then on a side stream
  // after the copy
  hipEvent_t ctl_event = nullptr, scan_event = nullptr;
  hipStream_t side_stream = nullptr;
  bool run_emit = false;  // take the emission path even for canonical terms
  bool run_counted = false;  // read the count before planning, even for small calls

  int read_ctl() {
    g_stats.host_syncs++;
    HIP_TRY(hipMemcpyAsync(hctl, dctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    g_prof.resolve();
    return PAULI_OK;
  }
  int zero_u32(void* p, size_t words) {
    if (!words) return PAULI_OK;
    const size_t blocks = (words + 255) / 256;
    LAUNCH("k_fill_u32", k_fill_u32, blocks, 256, (uint32_t*)p, 0u, words);
    return PAULI_OK;
  }
  int set_u64(unsigned long long* dst, unsigned long long v) {
    // small host->device update of the control block (not used under capture)
    g_stats.host_syncs++;
    HIP_TRY(hipMemcpyAsync(dst, &v, sizeof(v), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return PAULI_OK;
  }

  template <int W, bool F32>
  int run(Call& c);
};

int ws_short(Arena& ar, pauli_ws* ws) {
  ws->required = ar.need + (1 << 20);
  return PAULI_EWORKSPACE;
}

template <int W, bool F32>
int Engine::run(Call& c) {
  const size_t KB = sizeof(Key<W>);
  const size_t RB = sizeof(Rec<W, F32>);
  ar->bottom = 0;
  const size_t top0 = ar->top;
  memset(&g_stats, 0, sizeof(g_stats));
  // translation-symmetric commutator: H = sum_k T_k(H0), H0 listed over its
  // N translations (entry h N + k), then the plain commutator with every
  // product string replaced by its orbit representative
  if (c.ts && c.has_comm && c.H.n > 0) {
    const int64_t nf = c.H.n * c.ts;
    uint64_t* hx = (uint64_t*)ar->take((size_t)nf * 8 * W);
    uint64_t* hz = (uint64_t*)ar->take((size_t)nf * 8 * W);
    double2* hc = (double2*)ar->take((size_t)nf * sizeof(double2));
    if (ar->short_) return PAULI_EWORKSPACE;
    LAUNCH("k_ts_expand", (k_ts_expand<W>), (nf + 255) / 256, 256, c.H.x, c.H.z, c.H.cap,
           (const double2*)c.H.c, c.H.n, c.ts, hx, hz, hc);
    c.H.x = hx;
    c.H.z = hz;
    c.H.c = hc;
    c.H.n = nf;
    c.H.cap = nf;
  }
  // ----- inputs --------------------------------------------------------------
  const bool comm = c.has_comm && c.H.n > 0 && c.O.n > 0;
  int64_t tstart[MAX_TERMS + 1];
  tstart[0] = 0;
  for (int t = 0; t < c.n_terms; t++) tstart[t + 1] = tstart[t] + c.T[t].n;
  const int64_t nterm_rec = tstart[c.n_terms];
  const pauli_trunc* tr = c.trunc;
  const pauli_op* keep = tr ? tr->keep : nullptr;
  const int64_t n_keep = keep ? keep->size : 0;
  if (n_keep > 65536) return PAULI_EINVAL;
  if (keep && words_of(keep->n_qubits) != W) return PAULI_EINVAL;

  // every string's contributions must fit one merge bucket
  if (comm && c.H.n + c.n_terms + 8 > merge_cap<W>()) {
    g_last_error = "H has more strings than one merge bucket holds";
    return PAULI_EINVAL;
  }
  int comm_rows = 0, term_rows = 0;
  plan_rows(comm, c.O.n, nterm_rec, &comm_rows, &term_rows);
  const int rows = comm_rows + term_rows;

  Bufs1<W> b1;
  take_bufs1<W>(*ar, comm, c.H.n, n_keep, rows, b1);
  dctl = b1.dctl;
  uint64_t* Hk = b1.Hk;
  uint32_t* Hidx = b1.Hidx;
  uint32_t* hstart = b1.hstart;
  int* hspan = b1.hspan;
  Key<W>* keep_mk = b1.keep_mk;
  uint32_t* counts = b1.counts;
  uint32_t* bin_total = b1.bin_total;
  uint32_t* bin_base = b1.bin_base;
  uint32_t* hist0 = b1.hist0;
  uint32_t* histL[2] = {b1.histL[0], b1.histL[1]};
  uint32_t* hsum = b1.hsum;
  uint32_t* h0sum = b1.h0sum;
  unsigned long long* psum = b1.psum;
  if (ar->short_) return PAULI_EWORKSPACE;
  if (!hctl) TRY(host_ctl(&hctl));
  // the control block starts at zero (cleared by k_prep_h when there is one)
  if (!comm || rows == 0) TRY(zero_u32(dctl, sizeof(Ctl) / 4));

  auto write_empty = [&]() -> int {
    if (c.out.to_arena) {
      c.out.arena_op = OpV();
      c.out.arena_op.W = W;
      c.out.arena_op.f32 = c.out.f32;
    } else {
      c.out.user->size = 0;
    }
    return PAULI_OK;
  };
  if (rows == 0) {
    if (c.mode == M_LANCZOS) {
      if (c.b_out) *c.b_out = 0.0;
      write_empty();
      return PAULI_BREAKDOWN;
    }
    return write_empty();
  }
  if (comm) {
    LAUNCH("k_prep_h", (k_prep_h<W>), 1, 1024, c.H.x, c.H.z, c.H.cap, (int)c.H.n, Hk, Hidx,
           hstart, hspan, (uint32_t*)dctl, (uint32_t)(sizeof(Ctl) / 4));
  }
  if (n_keep) {
    LAUNCH("k_mix_keys", (k_mix_keys<W>), (n_keep + 255) / 256, 256, keep->x, keep->z,
           keep->capacity, n_keep, keep_mk, &dctl->bad_keep);
  }

  // ----- canonical terms: every bucket merged straight from its term runs ---
  // A linear combination with no commutator, no list term and one group per
  // term needs no emission when each term is in canonical order: the strings
  // of a hash bucket (top F bits of the mixed key) are one contiguous run of
  // every term.  Terms the engine wrote are canonical; the others are checked
  // on the device, and when one is out of order the merges leave every bucket
  // empty and the call is redone by emission (run_emit), as it is when strings
  // crowd one bucket beyond the merge's capacity.
  unsigned long long pe_all = 0;
  bool planned = false;  // one pass planned from the sizes alone (no count read)
  bool scattered = false;  // one pass over 2^14 bins scattered before the count was read
  const bool want_select = tr && tr->max_strings > 0;
  Bufs2 b2;
  MergeArgs ma;
  uint32_t nbk = 0;  // buckets written so far
  int npass = 1;
  auto merge_common = [&]() {
    memset(&ma, 0, sizeof(ma));
    for (int g = 0; g < c.n_groups; g++) {
      ma.alpha[g] = c.groups[g].alpha;
      ma.alpha_kind[g] = c.groups[g].divide ? A_DIV : alpha_kind(c.groups[g].alpha);
      ma.gkind[g] = c.groups[g].kind;
    }
    ma.mode = c.mode;
    ma.single = (c.n_groups == 1 && c.groups[0].kind != G_SUM_KAHAN32) ? 1 : 0;
    ma.round32 = c.round32 ? 1 : 0;
    ma.max_len = tr ? tr->max_len : 0;
    ma.use_eps = (tr && tr->coef_eps > 0.0) ? 1 : 0;
    ma.eps2 = tr ? tr->coef_eps * tr->coef_eps : 0.0;
    ma.keep_mk = keep_mk;
    ma.n_keep = (int)n_keep;
    ma.uk = b2.uk;
    ma.uc = b2.uc;
    ma.b_ubase = b2.b_ubase;
    ma.b_slots = b2.b_slots;
    ma.b_surv = b2.b_surv;
    ma.b_keep = b2.b_keep;
    ma.b_unique = b2.b_unique;
    ma.hist0 = hist0;
    ma.norm_part = b2.norm_part;
    ma.ctl = dctl;
    ma.defer = nullptr;
  };
  bool direct = !run_emit && !comm && c.n_terms > 0 && !c.ts && !c.product &&
                nterm_rec < ((int64_t)1 << 31);
  for (int t = 0; t < c.n_terms && direct; t++) {
    direct = !c.tlist[t];
    for (int u = 0; u < t; u++) direct = direct && c.tgroup[u] != c.tgroup[t];
  }
  if (direct) {
    // 2^F buckets of at most 0.85 of the small merge's capacity on average
    constexpr int SCAP = small_merge_cap<W, F32>();
    int F = 0;
    while (F < DIRECT_MAX_F && (double)nterm_rec > std::ldexp(0.85 * SCAP, F)) F++;
    const uint32_t nb = 1u << F;
    uint32_t* tbounds = (uint32_t*)ar->take((size_t)c.n_terms * (nb + 1) * 4);
    take_bufs2<W, F32>(*ar, (size_t)nterm_rec, false, false, nb, want_select, b2, false);
    if (ar->short_) return PAULI_EWORKSPACE;
    TermView tv;
    memset(&tv, 0, sizeof(tv));
    tv.n_terms = c.n_terms;
    tv.F = F;
    tv.bounds = tbounds;
    for (int t = 0; t < c.n_terms; t++) {
      const OpV& T = c.T[t];
      tv.tx[t] = T.x;
      tv.tz[t] = T.z;
      tv.tcap[t] = T.cap;
      tv.tn[t] = T.n;
      tv.tc[t] = T.c;
      tv.tf32[t] = T.f32;
      tv.tgroup[t] = (uint32_t)c.tgroup[t];
      if (!T.canon && T.n > 1)
        LAUNCH("k_check_sorted", (k_check_sorted<W>),
               (int)std::min<int64_t>((T.n + 255) / 256, 4096), 256, T.x, T.z, T.cap, T.n,
               &dctl->unsorted);
    }
    const int64_t nbounds = (int64_t)c.n_terms * (nb + 1);
    LAUNCH("k_term_bounds", (k_term_bounds<W>), (nbounds + 255) / 256, 256, tv, tbounds);
    TRY(zero_u32(hist0, (size_t)HREP * SEL0_BINS));
    merge_common();
    ma.tv = tv;
    ma.nbins_log = F;
    ma.digit_shift = F;
    ma.defer = b1.defer;
    // buckets above the small variant's capacity go to the full-size one
    LAUNCH("k_merge_small", (k_merge<W, F32, MERGE_SMALL_THREADS, SCAP, MERGE_SMALL, true>), nb,
           MERGE_SMALL_THREADS, ma);
    LAUNCH("k_merge_deferred",
           (k_merge<W, F32, MERGE_THREADS, merge_cap<W>(), MERGE_LIST, true>),
           std::min<uint32_t>(nb, 512), MERGE_THREADS, ma);
    nbk = nb;
    pe_all = (unsigned long long)nterm_rec;
  }
  if (!direct) {
    EmitArgs ea;
    memset(&ea, 0, sizeof(ea));
    ea.Hk = Hk;
    ea.Hidx = Hidx;
    ea.hstart = hstart;
    ea.hspan = hspan;
    ea.Hc = comm ? (const double2*)c.H.c : nullptr;
    ea.nH = comm ? (int)c.H.n : 0;
    ea.has_comm = comm ? 1 : 0;
    ea.product = c.product ? 1 : 0;
    ea.ts_n = c.ts;
    ea.comm_rows = comm_rows;
    ea.comm_group = (uint32_t)c.comm_group;
    if (comm) {
      ea.Ox = c.O.x;
      ea.Oz = c.O.z;
      ea.Ocap = c.O.cap;
      ea.nO = c.O.n;
      ea.Oc = c.O.c;
    }
    ea.n_terms = c.n_terms;
    ea.term_rows = term_rows;
    for (int t = 0; t < c.n_terms; t++) {
      ea.tx[t] = c.T[t].x;
      ea.tz[t] = c.T[t].z;
      ea.tcap[t] = c.T[t].cap;
      ea.tc[t] = c.T[t].c;
      ea.tf32[t] = c.T[t].f32;
      ea.tgroup[t] = (uint32_t)c.tgroup[t];
      ea.tlist[t] = c.tlist[t];
    }
    for (int t = 0; t <= c.n_terms; t++) ea.tstart[t] = tstart[t];
    ea.counts = counts;
    ea.bin_base = bin_base;
    ea.max_len = (c.mode == M_PLAIN && tr) ? tr->max_len : 0;

    // 2^nbl hash bins per pass: NBINS_LOG while the call fits one pass,
    // NBINS_LOG_MP (twice the records per pass) when it needs several, and
    // NBINS_LOG_SMALL for calls of at most 2^18 records even if every pair
    // emits one (the per-call bin tables then cost a sixteenth)
    int nbl = NBINS_LOG;
    const unsigned long long rec_bound =
        (comm ? (unsigned long long)c.H.n * (unsigned long long)c.O.n : 0ull) +
        (unsigned long long)nterm_rec;
    if (rec_bound <= (1ull << (NBINS_LOG_SMALL + 8))) nbl = NBINS_LOG_SMALL;
    auto count_pass = [&](int pass_bits, uint32_t pass_id, bool read = true,
                          unsigned long long spec_cap = 0ull) -> int {
      ea.pass_bits = pass_bits;
      ea.pass_id = pass_id;
      // the first count pass of a merge sequence also clears the level-0 |c|^2 histogram
      uint32_t* zero = pass_id == 0 ? hist0 : (uint32_t*)nullptr;
      const uint32_t nzero = pass_id == 0 ? (uint32_t)(HREP * SEL0_BINS) : 0u;
      if (nbl == NBINS_LOG_SMALL) {
        constexpr int NBS = 1 << NBINS_LOG_SMALL;
        LAUNCH("k_emit_count", (k_emit<W, F32, false, NBINS_LOG_SMALL>), rows, EMIT_THREADS, ea);
        if (rows <= SMALL_SCAN_ROWS) {
          LAUNCH("k_scan_small", k_scan_small, HREP, 1024, counts, rows, bin_base, dctl, zero,
                 nzero);
        } else {
          LAUNCH("k_scan_cols", k_scan_cols, NBS / SC_COLS, SC_COLS * SC_NSEG, counts, rows,
                 bin_total, dctl, NBS);
          LAUNCH("k_scan_bins", k_scan_bins<NBINS_LOG_SMALL>, 1, 1024, bin_total, bin_base, dctl,
                 zero, nzero);
        }
      } else if (nbl == NBINS_LOG) {
        LAUNCH("k_emit_count", (k_emit<W, F32, false, NBINS_LOG>), rows, EMIT_THREADS, ea);
        LAUNCH("k_scan_cols", k_scan_cols, NBINS / SC_COLS, SC_COLS * SC_NSEG, counts, rows, bin_total, dctl, NBINS);
        LAUNCH("k_scan_bins", k_scan_bins<NBINS_LOG>, 1, 1024, bin_total, bin_base, dctl, zero,
               nzero, spec_cap, (unsigned int)merge_cap<W>());
      } else {
        LAUNCH("k_emit_count", (k_emit<W, F32, false, NBINS_LOG_MP>), rows, EMIT_THREADS, ea);
        LAUNCH("k_scan_cols", k_scan_cols, NBINS_MP / SC_COLS, SC_COLS * SC_NSEG, counts, rows, bin_total, dctl,
               NBINS_MP);
        LAUNCH("k_scan_bins", k_scan_bins<NBINS_LOG_MP>, 1, 1024, bin_total, bin_base, dctl, zero,
               nzero);
      }
      return read ? read_ctl() : PAULI_OK;
    };
    // source ids fold into the key bits implied by the bin unless an index
    // needs more than 11 bits (H above 2047 strings, canonicalisation lists)
    // (translation-symmetric calls carry (H entry, rotation) as the source id)
    // (7 bits over 2^10 bins)
    auto wide_for = [&](int bins_log) {
      const int64_t max_h = bins_log == NBINS_LOG_SMALL ? (1 << (NBINS_LOG_SMALL - 3)) - 1 : 2047;
      bool w = comm && (c.H.n > max_h || c.ts);
      for (int t = 0; t < c.n_terms; t++) w = w || c.tlist[t];
      return w;
    };
    // A call of at most 2^18 possible records runs one pass over 2^10 bins
    // planned from its sizes alone (records laid out at that bound, a fixed
    // bucket width), so the host reads nothing before the output size; the
    // count's bins are checked then, and a call whose strings crowd a bucket
    // is redone with the count read first.
    if (nbl == NBINS_LOG_SMALL && !run_counted) {
      TRY(count_pass(0, 0, false));
      const size_t mark_bottom = ar->bottom, mark_need = ar->need;
      take_bufs2<W, F32>(*ar, (size_t)std::max<unsigned long long>(rec_bound, 1),
                         wide_for(NBINS_LOG_SMALL), false, (1u << NBINS_LOG_SMALL) << 2,
                         want_select, b2);
      if (ar->short_) {
        // the workspace holds the exact layout only: read the count
        ar->bottom = mark_bottom;
        ar->need = mark_need;
        ar->short_ = false;
        run_counted = true;
        TRY(read_ctl());
      } else {
        planned = true;
      }
    } else if (nbl == NBINS_LOG && ctl_event &&
               rec_bound <= 7ull * (1ull << NBINS_LOG) * (unsigned long long)merge_cap<W>()) {
      // A call that may fit one pass over 2^14 bins (at most seven passes'
      // worth of possible records) is laid out for as many records as the
      // workspace holds beside the rest of that pass; the count's control
      // block goes to the host behind an event and the scatter is launched
      // at once, so the GPU does not wait for the host's plan.  The bin scan
      // makes the scatter stand down when the records do not fit the layout
      // or a bin exceeds the merge capacity; the host then plans from the
      // count it has read, as below.
      const bool w14 = wide_for(NBINS_LOG);
      const uint32_t mb = (1u << NBINS_LOG) << 2;
      const size_t per = RB + KB + sizeof(double2) + (w14 ? 4 : 0) + (want_select ? 12 : 0) +
                         (c.out.to_arena ? (size_t)(16 * W + 16) : 0);
      const size_t fixed = (size_t)mb * (9 * 4 + sizeof(double2) + (want_select ? 12 : 0)) +
                           ((size_t)64 << 10);
      const size_t used = align256(ar->bottom) + ar->top;
      const size_t avail = ar->cap > used + fixed ? ar->cap - used - fixed : 0;
      const unsigned long long cap_rec =
          std::min<unsigned long long>(rec_bound, (unsigned long long)(avail / per));
      const size_t mark_bottom = ar->bottom, mark_need = ar->need;
      if (cap_rec >= (1ull << 16))
        take_bufs2<W, F32>(*ar, (size_t)cap_rec, w14, false, mb, want_select, b2);
      if (cap_rec < (1ull << 16) || ar->short_) {
        ar->bottom = mark_bottom;
        ar->need = mark_need;
        ar->short_ = false;
        TRY(count_pass(0, 0));
      } else {
        TRY(count_pass(0, 0, false, cap_rec));
        // the copy runs on a side stream once the scan is done, beside the scatter
        HIP_TRY(hipEventRecord(scan_event, stream));
        HIP_TRY(hipStreamWaitEvent(side_stream, scan_event, 0));
        HIP_TRY(hipMemcpyAsync(hctl, dctl, sizeof(Ctl), hipMemcpyDeviceToHost, side_stream));
        HIP_TRY(hipEventRecord(ctl_event, side_stream));
        ea.recs = b2.recs;
        ea.rsrc_wide = b2.rsrc_wide;
        ea.wide = w14 ? 1 : 0;
        ea.skip = &dctl->spec_fail;
        LAUNCH("k_emit_scatter", (k_emit<W, F32, true, NBINS_LOG>), rows, EMIT_THREADS, ea);
        ea.skip = nullptr;
        g_stats.host_syncs++;
        HIP_TRY(hipEventSynchronize(ctl_event));
        if (!hctl->spec_fail) {
          scattered = true;  // the pass stands: layout and records are in place
        } else {
          ar->bottom = mark_bottom;
          ar->need = mark_need;
        }
      }
    } else {
      TRY(count_pass(0, 0));
    }
    if (!planned && nbl == NBINS_LOG_SMALL && hctl->maxg[0] > (unsigned int)merge_cap<W>()) {
      // a small call whose records crowd one bin: count again over 2^14 bins
      nbl = NBINS_LOG;
      TRY(count_pass(0, 0));
    }
    if (!planned && hctl->bad_keep) return PAULI_EINVAL;
    if (!planned && (hctl->overflow & 2u)) {
      g_last_error = "more than 2^32 records in one pass";
      return PAULI_EINTERNAL;
    }
    pe_all = planned ? rec_bound : hctl->pe_total;
    // passes over disjoint hash ranges keep every bucket within the merge capacity; the
    // largest bin does not always halve with each extra pass bit (all records
    // of one string share a bin), so a pass that still overflows restarts the
    // loop with one more pass bit
    // the count pass measured every bin exactly
    int pass_bits = nbl == NBINS_LOG_SMALL ? 0 : plan_pass_bits<W>(hctl->maxg[0], &nbl);
    // Several passes bin each partition over 2^14 instead of 2^15 bins when
    // the 2^14 bins are expected to stay within 0.8 of the merge's capacity
    // (the merge then takes single bins where it would take pairs of 2^15
    // bins): half the destinations and count rows for the pass binning, and
    // its 64 KB bin table lets two blocks share a CU.
    int pnbl = nbl;  // bins per pass of the merge (and of the pass binning)
    if (!planned && nbl == NBINS_LOG_MP && pass_bits > 0 &&
        (double)hctl->maxg[0] <= std::ldexp(0.8 * merge_cap<W>(), pass_bits))
      pnbl = NBINS_LOG;
    const int table_bits = std::min(pass_bits + 2, MAX_PASS_BITS);
    const size_t ptot = (size_t)std::max<unsigned long long>(pe_all, 1);
    const uint32_t max_buckets = (uint32_t)(1u << nbl) << table_bits;
    // ----- records, U, bucket tables, candidate lists -------------------------
    const bool wide = wide_for(nbl);
    const bool partitioned = nbl == NBINS_LOG_MP;
    if (!planned && !scattered) {
      take_bufs2<W, F32>(*ar, ptot, wide, partitioned, max_buckets, want_select, b2);
      if (ar->short_) return PAULI_EWORKSPACE;
    }
    void* recs = b2.recs;
    uint32_t* rsrc_wide = b2.rsrc_wide;
    void* precs = b2.precs;
    uint32_t* ptop = b2.ptop;
    uint32_t* psrc = b2.psrc;
    uint32_t* pbase = b2.pbase;
    uint32_t* scounts = b2.scounts;
    void* uk = b2.uk;
    double2* uc = b2.uc;
    uint32_t* b_ubase = b2.b_ubase;
    uint32_t* b_slots = b2.b_slots;
    uint32_t* b_surv = b2.b_surv;
    uint32_t* b_keep = b2.b_keep;
    uint32_t* b_unique = b2.b_unique;
    uint32_t* b_abv = b2.b_abv;
    uint32_t* b_bcnt = b2.b_bcnt;
    uint32_t* b_obase = b2.b_obase;
    double2* norm_part = b2.norm_part;
    uint32_t* const* cand = b2.cand;
    uint32_t* const* ccnt = b2.ccnt;

    merge_common();
    ma.bin_base = bin_base;
    ma.recs = recs;
    ma.rsrc_wide = rsrc_wide;
    ma.wide = wide ? 1 : 0;

    ea.recs = recs;
    ea.rsrc_wide = rsrc_wide;
    ea.wide = wide ? 1 : 0;
    nbk = 0;  // buckets written so far
    npass = 1 << pass_bits;
    // the first count pass's prefixes (in `counts`) and bin totals (in
    // bin_total) serve the first partitioning only
    bool first_counts = pe_all < 0xFFFFFFFFull;
    for (bool done = false; !done;) {
      done = true;
      nbk = 0;
      unsigned long long u_off = 0;  // U slots reserved by earlier passes
      npass = 1 << pass_bits;
      SplitArgs sp;
      memset(&sp, 0, sizeof(sp));
      if (pass_bits > 0) {
        // emit every record once, into the partitions of its top pass_bits bits
        ea.part = 1;
        ea.pass_bits = pass_bits;
        ea.pass_id = 0;
        ea.recs = precs;
        ea.ptop = ptop;
        ea.psrc = psrc;
        ea.part_F = pnbl + pass_bits;
        ea.bin_base = pbase;
        if (first_counts && pass_bits <= 10) {
          // partition prefixes summed from the first count pass's bins, kept
          // above its rows x NBINS entries: no second pass over the pairs
          uint32_t* pcounts = counts + (size_t)rows * NBINS;
          LAUNCH("k_part_from_bins", k_part_from_bins, rows + 1, 1024, counts, rows, pass_bits,
                 1 << PART_NBL, pcounts, bin_total);
          ea.counts = pcounts;
        } else {
          LAUNCH("k_emit_part_count", (k_emit<W, F32, false, PART_NBL>), rows, EMIT_THREADS, ea);
          LAUNCH("k_scan_cols", k_scan_cols, (1 << PART_NBL) / SC_COLS, SC_COLS * SC_NSEG, counts, rows, bin_total, dctl,
                 1 << PART_NBL);
        }
        LAUNCH("k_scan_part", k_scan_part, 1, 1024, bin_total, npass, pbase, (1 << PART_NBL) + 1,
               dctl);
        LAUNCH("k_emit_part_scatter", (k_emit<W, F32, true, PART_NBL>), rows, EMIT_THREADS, ea);
        ea.counts = counts;
        first_counts = false;  // bin_total now holds partition, then split, totals
        ea.part = 0;
        ea.recs = recs;
        ea.bin_base = bin_base;
        sp.precs = precs;
        sp.ptop = ptop;
        sp.psrc = psrc;
        sp.pbase = pbase;
        sp.pass_bits = pass_bits;
        sp.wide = wide ? 1 : 0;
        sp.counts = scounts;
        sp.bin_base = bin_base;
        sp.recs = recs;
        sp.rsrc_wide = rsrc_wide;
      }
      for (int p = 0; p < npass; p++) {
        if (pass_bits > 0) {
          // bin partition p: histogram, scans (and the host check below)
          sp.part = (uint32_t)p;
          uint32_t* zero = p == 0 ? hist0 : (uint32_t*)nullptr;
          const uint32_t nzero = p == 0 ? (uint32_t)(HREP * SEL0_BINS) : 0u;
          if (pnbl == NBINS_LOG) {
            LAUNCH("k_split_count", (k_split<W, F32, false, NBINS_LOG>), SPLIT_ROWS, 1024, sp);
            LAUNCH("k_scan_cols", k_scan_cols, NBINS / SC_COLS, SC_COLS * SC_NSEG, scounts,
                   SPLIT_ROWS, bin_total, dctl, NBINS);
            LAUNCH("k_scan_bins", k_scan_bins<NBINS_LOG>, 1, 1024, bin_total, bin_base, dctl, zero,
                   nzero);
          } else {
            LAUNCH("k_split_count", (k_split<W, F32, false, NBINS_LOG_MP>), SPLIT_ROWS, 1024, sp);
            LAUNCH("k_scan_cols", k_scan_cols, NBINS_MP / SC_COLS, SC_COLS * SC_NSEG, scounts,
                   SPLIT_ROWS, bin_total, dctl, NBINS_MP);
            LAUNCH("k_scan_bins", k_scan_bins<NBINS_LOG_MP>, 1, 1024, bin_total, bin_base, dctl,
                   zero, nzero);
          }
          TRY(read_ctl());
        } else if (nbl == NBINS_LOG_MP) {
          // one pass at NBINS_LOG_MP bins: count again at that bin count; this
          // overwrites the first count pass's NBINS_LOG-bin prefixes and totals
          TRY(count_pass(pass_bits, (uint32_t)p));
          first_counts = false;
        }
        if (planned) {
          // buckets of 2^g bins whose mean stays within 0.85 of the small
          // merge's capacity even if every possible record is emitted; the
          // merges and the deferral list take whatever arrives, and a bucket
          // above the full-size merge's capacity sends the call round again
          constexpr int SCAP = small_merge_cap<W, F32>();
          int g_log = 4;
          while (g_log > 0 &&
                 (double)pe_all > std::ldexp(0.85 * SCAP, NBINS_LOG_SMALL - g_log))
            g_log--;
          LAUNCH("k_emit_scatter", (k_emit<W, F32, true, NBINS_LOG_SMALL>), rows, EMIT_THREADS, ea);
          ma.g_log = g_log;
          ma.nbins_log = nbl;
          ma.digit_shift = nbl - g_log;
          ma.pass_bits = 0;
          ma.pass_id = 0;
          ma.u_off = 0;
          ma.bucket_off = 0;
          const uint32_t nb_pass = (uint32_t)((1u << nbl) >> g_log);
          ma.defer = b1.defer;
          LAUNCH("k_merge_small", (k_merge<W, F32, MERGE_SMALL_THREADS, SCAP, MERGE_SMALL>),
                 nb_pass, MERGE_SMALL_THREADS, ma);
          // deferrals are rare here: a few blocks loop over the list
          LAUNCH("k_merge_deferred", (k_merge<W, F32, MERGE_THREADS, merge_cap<W>(), MERGE_LIST>),
                 std::min<uint32_t>(nb_pass, 16), MERGE_THREADS, ma);
          nbk = nb_pass;
          continue;
        }
        if (pass_bits > 0 && p == 0 && hctl->part_total != pe_all) {
          char msg[160];
          snprintf(msg, sizeof(msg), "partitions hold %llu records, the count pass %llu",
                   (unsigned long long)hctl->part_total, pe_all);
          g_last_error = msg;
          return PAULI_EINTERNAL;
        }
        const unsigned long long pe = hctl->pe_total;
        if (hctl->maxg[0] > (unsigned int)merge_cap<W>()) {
          if (pass_bits >= table_bits) {
            char msg[256];
            snprintf(msg, sizeof(msg),
                     "hash bucket above merge capacity: pass %d of %d, largest bin %u, "
                     "records in pass %llu, records in all passes %llu",
                     p, npass, hctl->maxg[0], (unsigned long long)pe, pe_all);
            g_last_error = msg;
            return PAULI_EINTERNAL;
          }
          pass_bits++;
          done = false;
          break;
        }
        int g_log = 4;
        while (g_log > 0 && hctl->maxg[g_log] > (unsigned int)merge_cap<W>()) g_log--;
        if (pe == 0) continue;
        if (pass_bits > 0 && pnbl == NBINS_LOG)
          LAUNCH("k_split_scatter", (k_split<W, F32, true, NBINS_LOG>), SPLIT_ROWS, 1024, sp);
        else if (pass_bits > 0)
          LAUNCH("k_split_scatter", (k_split<W, F32, true, NBINS_LOG_MP>), SPLIT_ROWS, 1024, sp);
        else if (scattered)
          ;  // launched before the count was read
        else if (nbl == NBINS_LOG_SMALL)
          LAUNCH("k_emit_scatter", (k_emit<W, F32, true, NBINS_LOG_SMALL>), rows, EMIT_THREADS, ea);
        else if (nbl == NBINS_LOG)
          LAUNCH("k_emit_scatter", (k_emit<W, F32, true, NBINS_LOG>), rows, EMIT_THREADS, ea);
        else
          LAUNCH("k_emit_scatter", (k_emit<W, F32, true, NBINS_LOG_MP>), rows, EMIT_THREADS, ea);
        ma.g_log = g_log;
        ma.nbins_log = pnbl;
        ma.digit_shift = pass_bits + pnbl - g_log;
        ma.pass_bits = pass_bits;
        ma.pass_id = (uint32_t)p;
        ma.u_off = u_off;
        ma.bucket_off = nbk;
        const uint32_t nb_pass = (uint32_t)((1u << pnbl) >> g_log);
        // Buckets up to the small variant's capacity run three to a CU: all
        // of them when the largest bucket fits; when most do, the full-size
        // merge takes the others from a deferral list; else the full-size merge
        // takes every bucket.
        constexpr int SCAP = small_merge_cap<W, F32>();
        const unsigned int big = hctl->maxg[g_log];
        ma.defer = b1.defer;
        if (big <= (unsigned int)SCAP) {
          LAUNCH("k_merge_small", (k_merge<W, F32, MERGE_SMALL_THREADS, SCAP, MERGE_SMALL>),
                 nb_pass, MERGE_SMALL_THREADS, ma);
        } else if (pe <= (unsigned long long)nb_pass * (SCAP * 7 / 8)) {
          LAUNCH("k_merge_small", (k_merge<W, F32, MERGE_SMALL_THREADS, SCAP, MERGE_SMALL>),
                 nb_pass, MERGE_SMALL_THREADS, ma);
          LAUNCH("k_merge_deferred", (k_merge<W, F32, MERGE_THREADS, merge_cap<W>(), MERGE_LIST>),
                 std::min<uint32_t>(nb_pass, 512), MERGE_THREADS, ma);
        } else {
          LAUNCH("k_merge", (k_merge<W, F32, MERGE_THREADS, merge_cap<W>(), MERGE_GRID>), nb_pass,
                 MERGE_THREADS, ma);
        }
        nbk += nb_pass;
        u_off += pe;
      }
    }
  }
  void* uk = b2.uk;
  double2* uc = b2.uc;
  uint32_t* b_ubase = b2.b_ubase;
  uint32_t* b_slots = b2.b_slots;
  uint32_t* b_surv = b2.b_surv;
  uint32_t* b_keep = b2.b_keep;
  uint32_t* b_unique = b2.b_unique;
  uint32_t* b_abv = b2.b_abv;
  uint32_t* b_bcnt = b2.b_bcnt;
  uint32_t* b_obase = b2.b_obase;
  double2* norm_part = b2.norm_part;
  uint32_t* const* cand = b2.cand;
  uint32_t* const* ccnt = b2.ccnt;
  g_stats.emitted = (int64_t)pe_all;
  g_stats.passes = npass;
  g_stats.buckets = (int32_t)nbk;
  if (nbk == 0) {
    TRY(read_ctl());
    if (hctl->overflow) {
      g_last_error = "merge bucket overflow";
      return PAULI_EINTERNAL;
    }
    g_stats.unique = 0;
    g_stats.survivors = 0;
    g_stats.output = 0;
    if (c.mode == M_LANCZOS) {
      if (c.b_out) *c.b_out = 0.0;
      write_empty();
      return PAULI_BREAKDOWN;
    }
    return write_empty();
  }

  // ----- Lanczos: b_n from the untruncated sum, then divide and filter -------
  const double lanczos_floor_b = 1e-13 * (c.b_prev > 1.0 ? c.b_prev : 1.0);
  if (c.mode == M_LANCZOS) {
    if (c.ts)
      LAUNCH("k_norm_bucket_ts", (k_norm_bucket_ts<W>), nbk, 256, b_ubase, b_slots, uk, uc,
             c.ts, norm_part);
    else
      LAUNCH("k_norm_bucket", k_norm_bucket, nbk, 256, b_ubase, b_slots, uc, norm_part);
    LAUNCH("k_reduce_dd", k_reduce_dd, 1, 1024, norm_part, nbk, &dctl->norm_hi);
    // b_n and the breakdown test are taken on the device (no read here); a
    // breakdown leaves nothing to keep, and the host reports it with the
    // output size
    ScaleArgs sa;
    memset(&sa, 0, sizeof(sa));
    sa.b_ubase = b_ubase;
    sa.b_slots = b_slots;
    sa.b_surv = b_surv;
    sa.b_keep = b_keep;
    sa.uk = uk;
    sa.uc = uc;
    sa.norm2 = &dctl->norm_hi;
    sa.floor_b = lanczos_floor_b;
    sa.round32 = c.out.f32;
    sa.max_len = ma.max_len;
    sa.use_eps = ma.use_eps;
    sa.eps2 = ma.eps2;
    sa.keep_mk = keep_mk;
    sa.n_keep = (int)n_keep;
    sa.hist0 = hist0;
    sa.ctl = dctl;
    LAUNCH("k_scale_filter", (k_scale_filter<W>), nbk, 256, sa);
  }

  // ----- top-M threshold, output offsets and write, decided on the device ---
  const int nchunk = (int)((nbk + SEL_CHUNK - 1) / SEL_CHUNK);
  Sel2Args s2;
  memset(&s2, 0, sizeof(s2));
  s2.b_ubase = b_ubase;
  s2.b_slots = b_slots;
  s2.b_abv = b_abv;
  s2.b_bcnt = b_bcnt;
  s2.uk = uk;
  s2.uc = uc;
  s2.keep_mk = keep_mk;
  s2.n_keep = (int)n_keep;
  s2.nbk = nbk;
  s2.ctl = dctl;
  if (want_select) {
    // the candidate lists of the multi-level select double as these lists
    s2.list0 = cand[1];
    s2.cc0 = ccnt[1];
    s2.listf = cand[0];
    s2.listfb = cand[2];
    s2.hist1 = histL[1];
  }
  PlanArgs pa;
  memset(&pa, 0, sizeof(pa));
  pa.b_slots = b_slots;
  pa.b_surv = b_surv;
  pa.b_keep = b_keep;
  pa.b_unique = b_unique;
  pa.nbk = nbk;
  pa.want_select = want_select ? 1 : 0;
  pa.max_strings = want_select ? (long long)tr->max_strings : 0;
  pa.hist0 = hist0;
  pa.hist1 = want_select ? histL[1] : nullptr;
  pa.psum = psum;
  pa.h0sum = h0sum;
  pa.ctl = dctl;
  LAUNCH("k_plan_sums", k_plan_sums, 3 * PLAN_PARTS, 1024, pa);
  LAUNCH("k_sel_plan", k_sel_plan, 1, 1024, pa);
  if (want_select) {
    LAUNCH("k_sel_pass1", (k_sel_pass1<W>), nchunk, 256, s2);
    LAUNCH("k_sel_pick1", k_sel_pick1, 1, 1024, histL[1], dctl);
    LAUNCH("k_sel_narrow", (k_sel_narrow<W>), nchunk, 256, s2);
    LAUNCH("k_sel_finish", (k_sel_finish<W>), 1, 1024, s2);
  }
  LAUNCH("k_scan_out", k_scan_out, 1, 1024, b_surv, b_keep, b_abv, b_bcnt, nbk, b_obase, dctl);

  WriteArgs wa;
  memset(&wa, 0, sizeof(wa));
  wa.b_ubase = b_ubase;
  wa.b_slots = b_slots;
  wa.b_obase = b_obase;
  wa.uk = uk;
  wa.uc = uc;
  wa.keep_mk = keep_mk;
  wa.n_keep = (int)n_keep;
  wa.ctl = dctl;
  wa.out_f32 = c.out.f32;
  if (c.out.to_arena) {
    // the output never exceeds the records emitted, nor max(M, |keep|) when
    // a top-M cut is asked for
    unsigned long long bound = pe_all;
    if (want_select)
      bound = std::min<unsigned long long>(
          bound, (unsigned long long)std::max<long long>((long long)tr->max_strings, n_keep));
    const size_t n = (size_t)std::max<unsigned long long>(bound, 1);
    uint64_t* ox = (uint64_t*)ar->take_top(n * 8 * W);
    uint64_t* oz = (uint64_t*)ar->take_top(n * 8 * W);
    void* oc = ar->take_top(n * (c.out.f32 ? 8 : 16));
    if (ar->short_) return PAULI_EWORKSPACE;
    c.out.arena_op.W = W;
    c.out.arena_op.f32 = c.out.f32;
    c.out.arena_op.canon = 1;
    c.out.arena_op.n = 0;
    c.out.arena_op.cap = (int64_t)n;
    c.out.arena_op.x = ox;
    c.out.arena_op.z = oz;
    c.out.arena_op.c = oc;
    wa.ox = ox;
    wa.oz = oz;
    wa.oc = oc;
    wa.ocap = (int64_t)n;
  } else {
    pauli_op* o = c.out.user;
    wa.ox = o->x;
    wa.oz = o->z;
    wa.oc = o->coef;
    wa.ocap = o->capacity;
  }
  LAUNCH("k_write_out", (k_write_out<W>), nchunk, 256, wa, nbk);
  TRY(read_ctl());
  if (direct && (hctl->unsorted || hctl->overflow)) {
    // a term out of canonical order (the buckets were left empty), or strings
    // crowded into one bucket beyond the merge's capacity: redo by emission,
    // whose hash-range passes split them
    ar->top = top0;
    run_emit = true;
    return run<W, F32>(c);
  }
  if (planned && (hctl->overflow || hctl->maxg[0] > (unsigned int)merge_cap<W>())) {
    // strings crowded into one bucket of the planned pass: redo with the
    // count read first, whose plan splits them
    ar->top = top0;
    run_counted = true;
    return run<W, F32>(c);
  }
  if (planned) {
    if (hctl->bad_keep) return PAULI_EINVAL;
    g_stats.emitted = (int64_t)hctl->pe_total;
  }
  if (direct && hctl->bad_keep) return PAULI_EINVAL;
  if (hctl->overflow) {
    g_last_error = "merge bucket overflow";
    return PAULI_EINTERNAL;
  }
  if (c.mode == M_LANCZOS) {
    const double b = std::sqrt(hctl->norm_hi);
    if (c.b_out) *c.b_out = b;
    if (!(b > lanczos_floor_b)) {
      write_empty();
      return PAULI_BREAKDOWN;
    }
  }
  g_stats.unique = (int64_t)hctl->u_unique;
  g_stats.survivors = (int64_t)hctl->surv_total;

  // Output size known: report it, or fall back to the host-driven multi-level
  // select when the device select stopped at a large group of equal |c|.
  auto finish_output = [&](unsigned long long nout) -> int {
    g_stats.output = (int64_t)nout;
    if ((unsigned long long)wa.ocap < nout) {
      if (c.out.to_arena) {
        g_last_error = "output above its bound";
        return PAULI_EINTERNAL;
      }
      c.out.user->size = (int64_t)nout;
      return PAULI_ECAPACITY;
    }
    if (c.out.to_arena) c.out.arena_op.n = (int64_t)nout;
    else c.out.user->size = (int64_t)nout;
    return PAULI_OK;
  };
  if (!hctl->deep) {
    if (hctl->sel_mode == S_THRESHOLD && !hctl->t_found) {
      g_last_error = "top-M threshold not found";
      return PAULI_EINTERNAL;
    }
    return finish_output(hctl->out_total);
  }

  // ----- fallback: threshold by as many 12-bit levels as the ties need ------
  const unsigned long long surv = hctl->surv_total, fk = hctl->keep_total;
  const unsigned long long nonkeep = surv - fk;
  int sel_mode = S_ALL;
  if (want_select) {
    const long long budget = (long long)tr->max_strings - (long long)fk;
    if (budget <= 0) sel_mode = fk == surv ? S_ALL : S_KEEP_ONLY;
    else if ((unsigned long long)budget >= nonkeep) sel_mode = S_ALL;
    else sel_mode = S_THRESHOLD;
    if (sel_mode == S_THRESHOLD) {
      SelArgs sa;
      memset(&sa, 0, sizeof(sa));
      sa.b_ubase = b_ubase;
      sa.b_slots = b_slots;
      sa.b_abv = b_abv;
      sa.b_bcnt = b_bcnt;
      sa.uk = uk;
      sa.uc = uc;
      sa.keep_mk = keep_mk;
      sa.n_keep = (int)n_keep;
      sa.nbk = nbk;
      sa.ctl = dctl;
      TRY(set_u64(&dctl->sel_K, (unsigned long long)budget));
      LAUNCH("k_hist_reduce", k_hist_reduce, SEL0_BINS / 256, 256, hist0, SEL0_BINS, hsum);
      LAUNCH("k_select", k_select, 1, 1024, hsum, SEL0_BINS, dctl);
      // level 1: full pass over U into list 0 (kept for the boundary count)
      TRY(zero_u32(histL[0], (size_t)HREP * SEL_BINS));
      sa.list_out = cand[0];
      sa.cc_out = ccnt[0];
      sa.hist = histL[0];
      LAUNCH("k_level1", (k_level1<W>), nbk, 256, sa);
      TRY(read_ctl());
      int in = 0;
      unsigned long long cnt = hctl->sel_count;
      if (cnt > FINISH_CAP) {
        int level = 1, hslot = 0;
        LAUNCH("k_hist_reduce", k_hist_reduce, SEL_BINS / 256, 256, histL[0], SEL_BINS, hsum);
        LAUNCH("k_select", k_select, 1, 1024, hsum, SEL_BINS, dctl);
        TRY(read_ctl());
        cnt = hctl->sel_count;
        while (cnt > FINISH_CAP) {
          if (level >= (64 + 128 * W) / 12) {
            g_last_error = "top-M select did not converge";
            return PAULI_EINTERNAL;
          }
          const int out = in == 1 ? 2 : 1;
          hslot ^= 1;
          TRY(zero_u32(histL[hslot], (size_t)HREP * SEL_BINS));
          sa.list_in = cand[in];
          sa.cc_in = ccnt[in];
          sa.list_out = cand[out];
          sa.cc_out = ccnt[out];
          sa.hist = histL[hslot];
          sa.level = level;
          LAUNCH("k_cand_level", (k_cand_level<W>), nbk, 256, sa);
          LAUNCH("k_hist_reduce", k_hist_reduce, SEL_BINS / 256, 256, histL[hslot], SEL_BINS,
                 hsum);
          LAUNCH("k_select", k_select, 1, 1024, hsum, SEL_BINS, dctl);
          TRY(read_ctl());
          cnt = hctl->sel_count;
          in = out;
          level++;
        }
        // narrow to the chosen bin of the last level
        const int out = in == 1 ? 2 : 1;
        sa.list_in = cand[in];
        sa.cc_in = ccnt[in];
        sa.list_out = cand[out];
        sa.cc_out = ccnt[out];
        sa.hist = nullptr;
        sa.level = level;
        LAUNCH("k_cand_level", (k_cand_level<W>), nbk, 256, sa);
        in = out;
      }
      sa.list_in = cand[in];
      sa.cc_in = ccnt[in];
      LAUNCH("k_finish", (k_finish<W>), 1, 1024, sa);
      sa.list_in = cand[0];
      sa.cc_in = ccnt[0];
      LAUNCH("k_count_boundary", (k_count_boundary<W>), nbk, 64, sa);
    }
  }
  LAUNCH("k_scan_buckets", k_scan_buckets, 1, 1024, b_surv, b_keep, b_abv, b_bcnt, nbk, sel_mode,
         b_obase, dctl);
  TRY(read_ctl());
  if (sel_mode == S_THRESHOLD && !hctl->t_found) {
    g_last_error = "top-M threshold not found";
    return PAULI_EINTERNAL;
  }
  const unsigned long long nout = hctl->out_total;
  if ((unsigned long long)wa.ocap >= nout && nout) {
    wa.sel_mode = sel_mode;
    LAUNCH("k_write", (k_write<W>), nbk, 256, wa);
    g_stats.host_syncs++;
    HIP_TRY(hipStreamSynchronize(stream));
    g_prof.resolve();
  }
  return finish_output(nout);
}

int dispatch(Engine& e, Call& c) {
  if (c.W == 1) return c.f32rec ? e.run<1, true>(c) : e.run<1, false>(c);
  if (c.W == 2) return c.f32rec ? e.run<2, true>(c) : e.run<2, false>(c);
  return PAULI_EINVAL;
}

// hctl: host copy of the control block (nullptr: this thread's pinned block)
int run_call(Arena& ar, pauli_ws* ws, void* stream, Call& c, Ctl* hctl = nullptr) {
  Engine e;
  e.ar = &ar;
  e.stream = (hipStream_t)stream;
  e.hctl = hctl;
  // the overlapped count read needs the pinned control block, two events and
  // a side stream (created once per thread, default priority); callers that
  // bring their own block get none of them
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (!hctl && (!t_side_stream || t_side_dev == dev)) {
    if (!t_side_stream) {
      HIP_TRY(hipEventCreateWithFlags(&t_ctl_event, hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&t_scan_event, hipEventDisableTiming));
      HIP_TRY(hipStreamCreateWithFlags(&t_side_stream, hipStreamNonBlocking));
      t_side_dev = dev;
    }
    e.ctl_event = t_ctl_event;
    e.scan_event = t_scan_event;
    e.side_stream = t_side_stream;
  }
  int rc = dispatch(e, c);
  if (rc == PAULI_EWORKSPACE || ar.short_) return ws_short(ar, ws);
  if (rc == PAULI_OK || rc == PAULI_BREAKDOWN) {
    // algorithmic bytes of the pass: inputs read, records written and read,
    // merged strings written and read, output written, at the record size
    int64_t inputs = (c.has_comm ? c.O.n : 0);
    for (int t = 0; t < c.n_terms; t++) inputs += c.T[t].n;
    const double rb = 16.0 * c.W + (c.f32rec ? 8.0 : 16.0);
    g_totals.calls++;
    g_totals.inputs += inputs;
    g_totals.emitted += g_stats.emitted;
    g_totals.unique += g_stats.unique;
    g_totals.output += g_stats.output;
    g_totals.alg_bytes += rb * (double)(inputs + 2 * g_stats.emitted + 2 * g_stats.unique +
                                        g_stats.output);
  }
  return rc;
}

Arena make_arena(pauli_ws* ws) {
  Arena a;
  a.base = (char*)ws->ptr;
  a.cap = ws->ptr ? ws->bytes : 0;
  return a;
}

OpV as_input(const OpV& v) { return v; }

// ---------------------------------------------------------------------------
// Workspace sizing without device work: the engine's own scratch layout on a
// dry arena, with the records at their bound from the sizes and bins assumed
// to fill evenly (largest bin at most 1.5 times the mean plus the records one
// string can collect).
// ---------------------------------------------------------------------------
struct DryCall {
  bool comm = false;
  int64_t nH = 0, nO = 0;   // commutator operands (nH after the translation expansion)
  int ts = 0;               // translation-symmetric sites (H0 listed over ts translates)
  int64_t nterm = 0;        // operator-term records
  int n_terms = 0;
  bool wide = false;        // source ids kept aside (long canonicalisation lists)
  int64_t n_keep = 0;
  bool select = false;
  int64_t out_arena = -1;   // >= 0: output rows taken from the top of the workspace
  bool out_f32 = false;
};

template <int W, bool F32>
void dry_call(Arena& ar, const DryCall& d, unsigned long long* pe_out) {
  ar.bottom = 0;
  int64_t nH = d.nH;
  if (d.ts && d.comm && d.nH > 0) {
    nH = d.nH * d.ts;
    ar.take((size_t)nH * 8 * W);
    ar.take((size_t)nH * 8 * W);
    ar.take((size_t)nH * sizeof(double2));
  }
  const bool comm = d.comm && nH > 0 && d.nO > 0;
  int comm_rows = 0, term_rows = 0;
  plan_rows(comm, d.nO, d.nterm, &comm_rows, &term_rows);
  Bufs1<W> b1;
  take_bufs1<W>(ar, comm, nH, d.n_keep, comm_rows + term_rows, b1);
  const unsigned long long pe =
      (comm ? (unsigned long long)nH * (unsigned long long)d.nO : 0ull) + (unsigned long long)d.nterm;
  if (pe_out) *pe_out = pe;
  const unsigned long long mx = pe * 3 / (2 * NBINS) + 1 + (comm ? nH : 0) + d.n_terms;
  int nbl = NBINS_LOG;
  const int pass_bits = plan_pass_bits<W>(mx, &nbl);
  const int table_bits = std::min(pass_bits + 2, MAX_PASS_BITS);
  const uint32_t max_buckets = (uint32_t)(1u << nbl) << table_bits;
  Bufs2 b2;
  // source ids aside as the engine decides (7-bit H indices over 2^10 bins)
  const int64_t max_h = pe <= (1ull << (NBINS_LOG_SMALL + 8)) ? (1 << (NBINS_LOG_SMALL - 3)) - 1 : 2047;
  take_bufs2<W, F32>(ar, (size_t)std::max<unsigned long long>(pe, 1), d.wide || (comm && (nH > max_h || d.ts)),
                     nbl == NBINS_LOG_MP, max_buckets, d.select, b2);
  if (d.out_arena >= 0) {
    const size_t n = (size_t)std::max<int64_t>(d.out_arena, 1);
    ar.take_top(n * 8 * W);
    ar.take_top(n * 8 * W);
    ar.take_top(n * (d.out_f32 ? 8 : 16));
  }
}

void dry(int W, bool f32rec, Arena& ar, const DryCall& d, unsigned long long* pe) {
  if (W == 1) f32rec ? dry_call<1, true>(ar, d, pe) : dry_call<1, false>(ar, d, pe);
  else f32rec ? dry_call<2, true>(ar, d, pe) : dry_call<2, false>(ar, d, pe);
}

// the output bound of a call emitting `pe` records under truncation t
int64_t out_bound(unsigned long long pe, const pauli_trunc* t) {
  unsigned long long b = pe;
  if (t && t->max_strings > 0) {
    const long long k = t->keep ? t->keep->size : 0;
    b = std::min<unsigned long long>(b, (unsigned long long)std::max<long long>(t->max_strings, k));
  }
  return (int64_t)std::max<unsigned long long>(b, 1);
}

int workspace_query(int op, const pauli_op* A, const pauli_op* B, const pauli_op* C,
                    const pauli_trunc* t, size_t* ws_bytes, int64_t* out_cap) {
  auto sz = [](const pauli_op* o) -> int64_t { return o ? std::max<int64_t>(o->size, 0) : 0; };
  const pauli_op* any = B ? B : A;
  if (!any || any->n_qubits < 1 || any->n_qubits > 128) return PAULI_EINVAL;
  const int W = words_of(any->n_qubits);
  const bool f32 = any->dtype == PAULI_C64K;
  const int64_t n_keep = (t && t->keep) ? t->keep->size : 0;
  const bool select = t && t->max_strings > 0;
  Arena ar;
  ar.dry = true;
  ar.cap = ~(size_t)0;
  unsigned long long pe = 0;
  int64_t cap = 1;
  DryCall d;
  d.n_keep = n_keep;
  d.select = select;
  switch (op) {
    case PAULI_Q_COMMUTATOR:
    case PAULI_Q_MULTIPLY:
    case PAULI_Q_COMMUTATOR_TS1D: {
      if (!A || !B) return PAULI_EINVAL;
      d.comm = true;
      d.nH = sz(A);
      d.nO = sz(B);
      d.ts = op == PAULI_Q_COMMUTATOR_TS1D ? B->n_qubits : 0;
      dry(W, f32, ar, d, &pe);
      cap = out_bound(pe, t);
      break;
    }
    case PAULI_Q_ADD: {
      if (!A || !B) return PAULI_EINVAL;
      d.nterm = sz(A) + sz(B);
      d.n_terms = 2;
      dry(W, A->dtype == PAULI_C64K && B->dtype == PAULI_C64K, ar, d, &pe);
      cap = out_bound(pe, t);
      break;
    }
    case PAULI_Q_TRUNCATE:
    case PAULI_Q_CANONICALIZE:
    case PAULI_Q_CANONICALIZE_TS1D: {
      if (!B) return PAULI_EINVAL;
      d.nterm = sz(B);
      d.n_terms = 1;
      d.wide = op != PAULI_Q_TRUNCATE;
      d.select = op == PAULI_Q_TRUNCATE && select;
      dry(W, f32, ar, d, &pe);
      cap = op == PAULI_Q_TRUNCATE ? out_bound(pe, t) : out_bound(pe, nullptr);
      break;
    }
    case PAULI_Q_LANCZOS:
    case PAULI_Q_LANCZOS_TS1D: {
      if (!A || !B) return PAULI_EINVAL;
      d.comm = true;
      d.nH = sz(A);
      d.nO = sz(B);
      d.ts = op == PAULI_Q_LANCZOS_TS1D ? B->n_qubits : 0;
      d.nterm = sz(C);
      d.n_terms = C ? 1 : 0;
      dry(W, f32, ar, d, &pe);
      cap = out_bound(pe, t);
      break;
    }
    case PAULI_Q_LANCZOS_REORTH: {
      if (!A || !B) return PAULI_EINVAL;
      DryCall d1;
      d1.comm = true;
      d1.nH = sz(A);
      d1.nO = sz(B);
      d1.nterm = sz(C);
      d1.n_terms = C ? 1 : 0;
      unsigned long long pe1 = 0;
      // O' at the top of the workspace, a bound without truncation
      d1.out_arena = (int64_t)std::max<unsigned long long>(
          (unsigned long long)d1.nH * (unsigned long long)d1.nO + (unsigned long long)d1.nterm, 1);
      dry(W, f32, ar, d1, &pe1);
      // projections: flags, results, partials, order keys of O_cur / O_prev
      ar.bottom = 0;
      ar.take(16);
      ar.take(6 * 16);
      ar.take((size_t)1024 * 16);
      ar.take((size_t)1024 * 16);
      ar.take((size_t)std::max<int64_t>(std::max(sz(B), sz(C)), 1) * 16 * W);
      d.nterm = d1.out_arena + sz(B) + sz(C);
      d.n_terms = 3;
      dry(W, false, ar, d, &pe);
      cap = out_bound(pe, t);
      break;
    }
    case PAULI_Q_RK4: {
      if (!A || !B) return PAULI_EINVAL;
      const int64_t nO = sz(B), nH = sz(A);
      int64_t S = nO, ksum = 0;
      for (int stage = 0; stage < 4; stage++) {
        DryCall dk;  // k = i [H, S], untruncated, at the top
        dk.comm = true;
        dk.nH = nH;
        dk.nO = S;
        const int64_t k = (int64_t)std::max<int64_t>(nH * S, 1);
        dk.out_arena = k;
        dry(W, false, ar, dk, nullptr);
        ksum += k;
        if (stage < 3) {
          DryCall ds;  // S = trunc(O + h k), at the top
          ds.nterm = nO + k;
          ds.n_terms = 2;
          ds.n_keep = n_keep;
          ds.select = select;
          ds.out_arena = out_bound((unsigned long long)(nO + k), t);
          dry(W, false, ar, ds, nullptr);
          S = ds.out_arena;
        }
      }
      d.nterm = nO + ksum;
      d.n_terms = 5;
      dry(W, false, ar, d, &pe);
      cap = out_bound(pe, t);
      break;
    }
    case PAULI_Q_REDUCTION: {
      // norm2, inner, trace, coefficients, norm2_ts1d: partials and order keys
      const int64_t n = std::max(sz(A), sz(B));
      ar.take(sizeof(Ctl));
      ar.take((size_t)std::max<int64_t>(n, 1) * 16 * W);
      ar.take((size_t)std::max<int64_t>(std::max(sz(A), sz(B)), 1) * 16);
      ar.take((size_t)1024 * 16);
      ar.take((size_t)1024 * 16);
      ar.take(32);
      cap = 0;
      break;
    }
    default:
      return PAULI_EINVAL;
  }
  // the engine adds the same margin when it reports a shortfall
  if (ws_bytes) *ws_bytes = ar.need + (1 << 20);
  if (out_cap) *out_cap = cap;
  return PAULI_OK;
}

// ---------------------------------------------------------------------------
// Scratch that needs no allocation: a file-scope device array (one copy per
// GPU, held until the process ends) for callers that cannot allocate.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): its device address on each GPU comes from
// hipGetSymbolAddress, taken once per device with that device current.
// ---------------------------------------------------------------------------
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)256 << 20;
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {nullptr};
// host copy of the control block for these calls (pageable: no host allocation)
thread_local Ctl t_static_hctl;

}  // namespace

__device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {
int static_scratch(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) {
    g_last_error = "device ordinal beyond the static scratch table";
    return PAULI_EINVAL;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p & 255)) {
      g_last_error = "static scratch address not 256-byte aligned";
      return PAULI_EINTERNAL;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PAULI_OK;
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* pauli_strerror(int status) {
  switch (status) {
    case PAULI_OK: return "ok";
    case PAULI_EINVAL: return "invalid argument";
    case PAULI_ECAPACITY: return "output capacity too small (size holds the requirement)";
    case PAULI_EWORKSPACE: return "workspace too small (ws->required holds the requirement)";
    case PAULI_BREAKDOWN: return "Lanczos breakdown: b_n is zero";
    case PAULI_EHIP: return "HIP runtime error";
    case PAULI_EINTERNAL: return "internal limit exceeded";
    default: return "unknown status";
  }
}

const char* pauli_last_error(void) { return g_last_error.c_str(); }

void pauli_last_stats(pauli_stats* out) {
  if (out) *out = g_stats;
}

void pauli_read_totals(pauli_totals* out, int reset) {
  if (out) *out = g_totals;
  if (reset) memset(&g_totals, 0, sizeof(g_totals));
}

void pauli_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  g_prof.on = on != 0;
  g_prof.acc.clear();
}

void pauli_profile_only(const char* names) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  g_prof.only.clear();
  if (!names) return;
  std::string cur;
  for (const char* q = names;; q++) {
    if (*q == ',' || *q == 0) {
      if (!cur.empty()) g_prof.only.insert(cur);
      cur.clear();
      if (*q == 0) break;
    } else {
      cur += *q;
    }
  }
}

size_t pauli_profile_read(char* buf, size_t len) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  std::string s;
  char line[256];
  for (auto& kv : g_prof.acc) {
    snprintf(line, sizeof(line), "%s %ld %.9f\n", kv.first.c_str(), kv.second.first,
             kv.second.second);
    s += line;
  }
  if (buf && len) {
    size_t n = std::min(len - 1, s.size());
    memcpy(buf, s.data(), n);
    buf[n] = 0;
  }
  return s.size() + 1;
}

int pauli_commutator(const pauli_op* H, const pauli_op* O, const pauli_trunc* t, pauli_op* out,
                     pauli_ws* ws, void* stream) {
  if (!ws || check_op(H, false) || check_op(O, false) || check_op(out, true)) return PAULI_EINVAL;
  if (H->n_qubits != O->n_qubits || out->n_qubits != O->n_qubits) return PAULI_EINVAL;
  if (H->dtype != PAULI_C128 || out->dtype != O->dtype) return PAULI_EINVAL;
  Arena ar = make_arena(ws);
  Call c;
  c.W = words_of(O->n_qubits);
  c.f32rec = O->dtype == PAULI_C64K;
  c.has_comm = true;
  c.H = view(H);
  c.O = view(O);
  c.comm_group = 0;
  c.n_groups = 1;
  c.groups[0].kind = c.f32rec ? G_SUM_KAHAN32 : G_SUM;
  c.trunc = t;
  c.out.user = out;
  c.out.f32 = out->dtype == PAULI_C64K;
  c.round32 = c.out.f32;
  return run_call(ar, ws, stream, c);
}

int pauli_commutator_noalloc(const pauli_op* H, const pauli_op* O, const pauli_trunc* t,
                             pauli_op* out, void* stream) {
  if (check_op(H, false) || check_op(O, false) || check_op(out, true)) return PAULI_EINVAL;
  if (H->n_qubits != O->n_qubits || out->n_qubits != O->n_qubits) return PAULI_EINVAL;
  if (H->dtype != PAULI_C128 || out->dtype != O->dtype) return PAULI_EINVAL;
  void* base = nullptr;
  TRY(static_scratch(&base));
  pauli_ws ws = {base, STATIC_SCRATCH_BYTES, 0};
  Arena ar = make_arena(&ws);
  Call c;
  c.W = words_of(O->n_qubits);
  c.f32rec = O->dtype == PAULI_C64K;
  c.has_comm = true;
  c.H = view(H);
  c.O = view(O);
  c.comm_group = 0;
  c.n_groups = 1;
  c.groups[0].kind = c.f32rec ? G_SUM_KAHAN32 : G_SUM;
  c.trunc = t;
  c.out.user = out;
  c.out.f32 = out->dtype == PAULI_C64K;
  c.round32 = c.out.f32;
  const int rc = run_call(ar, &ws, stream, c, &t_static_hctl);
  if (rc == PAULI_EWORKSPACE) {
    char msg[200];
    snprintf(msg, sizeof(msg),
             "the call needs %zu bytes of scratch; the static scratch holds %zu",
             ws.required, STATIC_SCRATCH_BYTES);
    g_last_error = msg;
  }
  return rc;
}

int pauli_multiply(const pauli_op* A, const pauli_op* B, const pauli_trunc* t, pauli_op* out,
                   pauli_ws* ws, void* stream) {
  if (!ws || check_op(A, false) || check_op(B, false) || check_op(out, true)) return PAULI_EINVAL;
  if (A->n_qubits != B->n_qubits || out->n_qubits != B->n_qubits) return PAULI_EINVAL;
  if (A->dtype != PAULI_C128 || out->dtype != B->dtype) return PAULI_EINVAL;
  Arena ar = make_arena(ws);
  Call c;
  c.W = words_of(B->n_qubits);
  c.f32rec = B->dtype == PAULI_C64K;
  c.has_comm = true;
  c.product = true;
  c.H = view(A);
  c.O = view(B);
  c.comm_group = 0;
  c.n_groups = 1;
  c.groups[0].kind = c.f32rec ? G_SUM_KAHAN32 : G_SUM;
  c.trunc = t;
  c.out.user = out;
  c.out.f32 = out->dtype == PAULI_C64K;
  c.round32 = c.out.f32;
  return run_call(ar, ws, stream, c);
}

int pauli_commutator_ts1d(const pauli_op* H0, const pauli_op* O, const pauli_trunc* t,
                          pauli_op* out, pauli_ws* ws, void* stream) {
  if (!ws || check_op(H0, false) || check_op(O, false) || check_op(out, true)) return PAULI_EINVAL;
  if (H0->n_qubits != O->n_qubits || out->n_qubits != O->n_qubits) return PAULI_EINVAL;
  if (H0->dtype != PAULI_C128 || out->dtype != O->dtype) return PAULI_EINVAL;
  Arena ar = make_arena(ws);
  Call c;
  c.W = words_of(O->n_qubits);
  c.f32rec = O->dtype == PAULI_C64K;
  c.has_comm = true;
  c.ts = O->n_qubits;
  c.H = view(H0);
  c.O = view(O);
  c.comm_group = 0;
  c.n_groups = 1;
  c.groups[0].kind = c.f32rec ? G_SUM_KAHAN32 : G_SUM;
  c.trunc = t;
  c.out.user = out;
  c.out.f32 = out->dtype == PAULI_C64K;
  c.round32 = c.out.f32;
  return run_call(ar, ws, stream, c);
}

int pauli_canonicalize_ts1d(const pauli_op* in, pauli_op* out, pauli_ws* ws, void* stream) {
  if (!ws || check_op(in, false) || check_op(out, true)) return PAULI_EINVAL;
  if (out->n_qubits != in->n_qubits) return PAULI_EINVAL;
  if (in->size >= ((int64_t)1 << GROUP_SHIFT)) return PAULI_EINVAL;
  Arena ar = make_arena(ws);
  Call c;
  c.W = words_of(in->n_qubits);
  c.f32rec = in->dtype == PAULI_C64K;
  c.ts = in->n_qubits;
  c.n_terms = 1;
  c.T[0] = view(in);
  c.tlist[0] = 1;
  c.n_groups = 1;
  c.groups[0].kind = G_SUM;
  c.out.user = out;
  c.out.f32 = out->dtype == PAULI_C64K;
  c.round32 = c.out.f32;
  return run_call(ar, ws, stream, c);
}

int pauli_norm2_ts1d(const pauli_op* A, double* out, pauli_ws* ws, void* stream_) {
  if (!ws || !out || check_op(A, false)) return PAULI_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  Arena ar = make_arena(ws);
  const int blocks = (int)std::min<int64_t>(std::max<int64_t>((A->size + 255) / 256, 1), 1024);
  double2* part = (double2*)ar.take((size_t)blocks * 16);
  double* res = (double*)ar.take(16);
  if (ar.short_) return ws_short(ar, ws);
  if (A->size == 0) {
    *out = 0.0;
    return PAULI_OK;
  }
  const int W = words_of(A->n_qubits), N = A->n_qubits;
  const bool f32 = A->dtype == PAULI_C64K;
  if (W == 1) {
    if (f32)
      LAUNCH("k_norm_part_ts", (k_norm_part_ts<1, true>), blocks, 256, A->x, A->z, A->capacity,
             A->coef, A->size, N, part);
    else
      LAUNCH("k_norm_part_ts", (k_norm_part_ts<1, false>), blocks, 256, A->x, A->z, A->capacity,
             A->coef, A->size, N, part);
  } else {
    if (f32)
      LAUNCH("k_norm_part_ts", (k_norm_part_ts<2, true>), blocks, 256, A->x, A->z, A->capacity,
             A->coef, A->size, N, part);
    else
      LAUNCH("k_norm_part_ts", (k_norm_part_ts<2, false>), blocks, 256, A->x, A->z, A->capacity,
             A->coef, A->size, N, part);
  }
  LAUNCH("k_reduce_dd", k_reduce_dd, 1, 1024, part, (uint32_t)blocks, res);
  double h[2];
  HIP_TRY(hipMemcpyAsync(h, res, 16, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  g_prof.resolve();
  *out = h[0];
  return PAULI_OK;
}

int pauli_trace(const pauli_op* A, double out[2], pauli_ws* ws, void* stream_) {
  if (!ws || !out || check_op(A, false)) return PAULI_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  Arena ar = make_arena(ws);
  double* res = (double*)ar.take(16);
  if (ar.short_) return ws_short(ar, ws);
  out[0] = 0.0;
  out[1] = 0.0;
  if (A->size == 0) return PAULI_OK;
  const int W = words_of(A->n_qubits);
  LAUNCH("k_fill_u32", k_fill_u32, 1, 256, (uint32_t*)res, 0u, (size_t)4);
  const int blocks = (int)std::min<int64_t>((A->size + 255) / 256, 4096);
  LAUNCH("k_trace", k_trace, blocks, 256, A->x, A->z, A->capacity, A->size, W,
         A->coef, A->dtype == PAULI_C64K ? 1 : 0, res);
  double h[2];
  HIP_TRY(hipMemcpyAsync(h, res, 16, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  g_prof.resolve();
  out[0] = h[0];
  out[1] = h[1];
  return PAULI_OK;
}

int pauli_add(const pauli_op* A, double ar_, double ai, const pauli_op* B, double br, double bi,
              const pauli_trunc* t, pauli_op* out, pauli_ws* ws, void* stream) {
  if (!ws || check_op(A, false) || check_op(B, false) || check_op(out, true)) return PAULI_EINVAL;
  if (A->n_qubits != B->n_qubits || out->n_qubits != A->n_qubits) return PAULI_EINVAL;
  Arena ar = make_arena(ws);
  Call c;
  c.W = words_of(A->n_qubits);
  c.f32rec = A->dtype == PAULI_C64K && B->dtype == PAULI_C64K;
  c.n_terms = 2;
  c.T[0] = view(A);
  c.T[1] = view(B);
  c.tgroup[0] = 0;
  c.tgroup[1] = 1;
  c.n_groups = 2;
  c.groups[0].alpha = make_double2(ar_, ai);
  c.groups[1].alpha = make_double2(br, bi);
  c.trunc = t;
  c.out.user = out;
  c.out.f32 = out->dtype == PAULI_C64K;
  c.round32 = c.out.f32;
  return run_call(ar, ws, stream, c);
}

int pauli_truncate(const pauli_op* in, const pauli_trunc* t, pauli_op* out, pauli_ws* ws,
                   void* stream) {
  if (!ws || check_op(in, false) || check_op(out, true)) return PAULI_EINVAL;
  if (out->n_qubits != in->n_qubits) return PAULI_EINVAL;
  Arena ar = make_arena(ws);
  Call c;
  c.W = words_of(in->n_qubits);
  c.f32rec = in->dtype == PAULI_C64K;
  c.n_terms = 1;
  c.T[0] = view(in);
  c.n_groups = 1;
  c.trunc = t;
  c.out.user = out;
  c.out.f32 = out->dtype == PAULI_C64K;
  c.round32 = c.out.f32;
  return run_call(ar, ws, stream, c);
}

int pauli_divide(const pauli_op* in, double b, pauli_op* out, pauli_ws* ws, void* stream) {
  if (!ws || check_op(in, false) || check_op(out, true)) return PAULI_EINVAL;
  if (out->n_qubits != in->n_qubits || !(std::isfinite(b) && b != 0.0)) return PAULI_EINVAL;
  Arena ar = make_arena(ws);
  Call c;
  c.W = words_of(in->n_qubits);
  c.f32rec = in->dtype == PAULI_C64K;
  c.n_terms = 1;
  c.T[0] = view(in);
  c.n_groups = 1;
  c.groups[0].alpha = make_double2(b, 0.0);
  c.groups[0].divide = true;
  c.out.user = out;
  c.out.f32 = out->dtype == PAULI_C64K;
  c.round32 = c.out.f32;
  return run_call(ar, ws, stream, c);
}

int pauli_canonicalize(const pauli_op* in, pauli_op* out, pauli_ws* ws, void* stream) {
  if (!ws || check_op(in, false) || check_op(out, true)) return PAULI_EINVAL;
  if (out->n_qubits != in->n_qubits) return PAULI_EINVAL;
  if (in->size >= ((int64_t)1 << GROUP_SHIFT)) return PAULI_EINVAL;
  Arena ar = make_arena(ws);
  Call c;
  c.W = words_of(in->n_qubits);
  c.f32rec = in->dtype == PAULI_C64K;
  c.n_terms = 1;
  c.T[0] = view(in);
  c.tlist[0] = 1;
  c.n_groups = 1;
  c.groups[0].kind = G_SUM;
  c.out.user = out;
  c.out.f32 = out->dtype == PAULI_C64K;
  c.round32 = c.out.f32;
  return run_call(ar, ws, stream, c);
}

// ts = N: translation-symmetric operators of the periodic chain (H holds H0,
// the operators orbit representatives), else 0.
static int lanczos_step(const pauli_op* H, const pauli_op* O_prev, const pauli_op* O_cur,
                        double b_prev, const pauli_trunc* t, int ts, pauli_op* O_next,
                        double* b_out, pauli_ws* ws, void* stream) {
  if (!ws || check_op(H, false) || check_op(O_cur, false) || check_op(O_next, true))
    return PAULI_EINVAL;
  if (O_prev && check_op(O_prev, false)) return PAULI_EINVAL;
  if (H->dtype != PAULI_C128 || O_next->dtype != O_cur->dtype) return PAULI_EINVAL;
  if (O_prev && O_prev->dtype != O_cur->dtype) return PAULI_EINVAL;
  if (H->n_qubits != O_cur->n_qubits || O_next->n_qubits != O_cur->n_qubits ||
      (O_prev && O_prev->n_qubits != O_cur->n_qubits))
    return PAULI_EINVAL;
  Arena ar = make_arena(ws);
  Call c;
  c.W = words_of(O_cur->n_qubits);
  c.f32rec = O_cur->dtype == PAULI_C64K;
  c.has_comm = true;
  c.ts = ts;
  c.H = view(H);
  c.O = view(O_cur);
  c.comm_group = 0;
  c.n_groups = 1;
  c.groups[0].kind = c.f32rec ? G_SUM_KAHAN32 : G_SUM;
  if (O_prev && O_prev->size > 0) {
    c.n_terms = 1;
    c.T[0] = view(O_prev);
    c.tgroup[0] = 1;
    c.n_groups = 2;
    c.groups[1].kind = G_TERM;
    c.groups[1].alpha = make_double2(-b_prev, 0.0);
  }
  c.mode = M_LANCZOS;
  c.trunc = t;
  c.out.user = O_next;
  c.out.f32 = O_next->dtype == PAULI_C64K;
  c.b_prev = b_prev;
  double b = 0.0;
  c.b_out = &b;
  int rc = run_call(ar, ws, stream, c);
  if (b_out) *b_out = b;
  return rc;
}

// Lanczos step with local re-orthogonalisation: O' = [H, O_cur] - b_prev O_prev
// (untruncated, FP64, at the top of the workspace), then
// O'' = O' - (<O_cur,O'>/<O_cur,O_cur>) O_cur - (<O_prev,O'>/<O_prev,O_prev>) O_prev
// with both coefficients taken from O' (inner products and norms summed in
// double-double, rounded once, divided in FP64), b_n = ||O''||,
// O_next = trunc(O'' / b_n).
static int lanczos_step_reorth(const pauli_op* H, const pauli_op* O_prev, const pauli_op* O_cur,
                               double b_prev, const pauli_trunc* t, pauli_op* O_next,
                               double* b_out, pauli_ws* ws, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  Arena ar = make_arena(ws);
  const int W = words_of(O_cur->n_qubits);
  const bool f32 = O_cur->dtype == PAULI_C64K;
  const bool has_prev = O_prev && O_prev->size > 0;
  double b = 0.0;
  // 1. O' in FP64 (the commutator in FP32 with compensated sums for PAULI_C64K)
  Call c1;
  c1.W = W;
  c1.f32rec = f32;
  c1.has_comm = true;
  c1.H = view(H);
  c1.O = view(O_cur);
  c1.n_groups = 1;
  c1.groups[0].kind = f32 ? G_SUM_KAHAN32 : G_SUM;
  if (has_prev) {
    c1.n_terms = 1;
    c1.T[0] = view(O_prev);
    c1.tgroup[0] = 1;
    c1.n_groups = 2;
    c1.groups[1].kind = G_TERM;
    c1.groups[1].alpha = make_double2(-b_prev, 0.0);
  }
  c1.out.to_arena = true;
  c1.out.f32 = 0;
  TRY(run_call(ar, ws, stream, c1));
  const OpV Op = c1.out.arena_op;
  // 2. projections of O' on O_cur and O_prev
  double2 alpha[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
  const pauli_op* V[2] = {O_cur, has_prev ? O_prev : nullptr};
  if (Op.n > 0) {
    ar.bottom = 0;
    unsigned int* bad = (unsigned int*)ar.take(16);
    double* res = (double*)ar.take(6 * 16);
    const int blocks = (int)std::min<int64_t>(std::max<int64_t>((Op.n + 255) / 256, 1), 1024);
    double2* pr = (double2*)ar.take((size_t)1024 * 16);  // partials of up to 1024 blocks
    double2* pi = (double2*)ar.take((size_t)1024 * 16);
    int64_t nk = 0;
    for (int k = 0; k < 2; k++)
      if (V[k]) nk = std::max<int64_t>(nk, V[k]->size);
    void* vmk = ar.take((size_t)std::max<int64_t>(nk, 1) * 16 * W);
    if (ar.short_) return ws_short(ar, ws);
    LAUNCH("k_fill_u32", k_fill_u32, 1, 256, (uint32_t*)bad, 0u, (size_t)4);
    for (int k = 0; k < 2; k++) {
      const pauli_op* v = V[k];
      if (!v || v->size == 0) continue;
      const int vb = (int)std::min<int64_t>((v->size + 255) / 256, 1024);
      const int vf32 = v->dtype == PAULI_C64K;
      // <O', V> = sum conj(o') v over common strings (V canonical: binary search)
      if (W == 1) {
        LAUNCH("k_mix_keys", k_mix_keys<1>, (v->size + 255) / 256, 256, v->x, v->z, v->capacity,
               v->size, (Key<1>*)vmk, bad);
        LAUNCH("k_inner_part", k_inner_part<1>, blocks, 256, Op.x, Op.z, Op.cap, Op.n, Op.c, 0,
               (const Key<1>*)vmk, v->size, v->coef, vf32, pr, pi);
      } else {
        LAUNCH("k_mix_keys", k_mix_keys<2>, (v->size + 255) / 256, 256, v->x, v->z, v->capacity,
               v->size, (Key<2>*)vmk, bad);
        LAUNCH("k_inner_part", k_inner_part<2>, blocks, 256, Op.x, Op.z, Op.cap, Op.n, Op.c, 0,
               (const Key<2>*)vmk, v->size, v->coef, vf32, pr, pi);
      }
      LAUNCH("k_reduce_dd", k_reduce_dd, 1, 1024, pr, (uint32_t)blocks, res + 6 * k);
      LAUNCH("k_reduce_dd", k_reduce_dd, 1, 1024, pi, (uint32_t)blocks, res + 6 * k + 2);
      // ||V||^2 (the partials reuse pr: same stream, after the reduction above)
      if (vf32)
        LAUNCH("k_norm_part", k_norm_part<true>, vb, 256, v->coef, v->size, pr);
      else
        LAUNCH("k_norm_part", k_norm_part<false>, vb, 256, v->coef, v->size, pr);
      LAUNCH("k_reduce_dd", k_reduce_dd, 1, 1024, pr, (uint32_t)vb, res + 6 * k + 4);
    }
    double h[12];
    unsigned int hbad = 0;
    HIP_TRY(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    g_prof.resolve();
    if (hbad) {
      g_last_error = "re-orthogonalisation needs canonical O_cur and O_prev";
      return PAULI_EINVAL;
    }
    for (int k = 0; k < 2; k++) {
      if (!V[k] || V[k]->size == 0) continue;
      const double n2 = h[6 * k + 4];
      // <V, O'> = conj(<O', V>), divided by <V, V>
      if (n2 > 0.0) alpha[k] = make_double2(h[6 * k] / n2, -h[6 * k + 2] / n2);
    }
  }
  // 3. O'' = O' - alpha_0 O_cur - alpha_1 O_prev, b_n, divide, truncate
  Call c2;
  c2.W = W;
  c2.f32rec = false;
  c2.n_terms = 0;
  c2.n_groups = 0;
  // a term with a zero coefficient only adds exact zeros: left out
  auto add_term = [&](const OpV& v, double2 al) {
    if (v.n == 0 || (al.x == 0.0 && al.y == 0.0)) return;
    c2.T[c2.n_terms] = v;
    c2.tgroup[c2.n_terms] = c2.n_groups;
    c2.groups[c2.n_groups].kind = G_TERM;
    c2.groups[c2.n_groups].alpha = al;
    c2.n_terms++;
    c2.n_groups++;
  };
  add_term(Op, make_double2(1.0, 0.0));
  for (int k = 0; k < 2; k++)
    if (V[k]) add_term(view(V[k]), make_double2(-alpha[k].x, -alpha[k].y));
  c2.mode = M_LANCZOS;
  c2.trunc = t;
  c2.out.user = O_next;
  c2.out.f32 = f32;
  c2.b_prev = b_prev;
  c2.b_out = &b;
  const int rc = run_call(ar, ws, stream, c2);
  if (b_out) *b_out = b;
  return rc;
}

int pauli_lanczos_step(const pauli_op* H, const pauli_op* O_prev, const pauli_op* O_cur,
                       double b_prev, const pauli_trunc* t, uint32_t flags, pauli_op* O_next,
                       double* b_out, pauli_ws* ws, void* stream) {
  if (flags & ~(uint32_t)PAULI_REORTH_LOCAL) return PAULI_EINVAL;
  if (!(flags & PAULI_REORTH_LOCAL))
    return lanczos_step(H, O_prev, O_cur, b_prev, t, 0, O_next, b_out, ws, stream);
  if (!ws || check_op(H, false) || check_op(O_cur, false) || check_op(O_next, true))
    return PAULI_EINVAL;
  if (O_prev && check_op(O_prev, false)) return PAULI_EINVAL;
  if (H->dtype != PAULI_C128 || O_next->dtype != O_cur->dtype) return PAULI_EINVAL;
  if (O_prev && O_prev->dtype != O_cur->dtype) return PAULI_EINVAL;
  if (H->n_qubits != O_cur->n_qubits || O_next->n_qubits != O_cur->n_qubits ||
      (O_prev && O_prev->n_qubits != O_cur->n_qubits))
    return PAULI_EINVAL;
  return lanczos_step_reorth(H, O_prev, O_cur, b_prev, t, O_next, b_out, ws, stream);
}

int pauli_lanczos_step_ts1d(const pauli_op* H0, const pauli_op* O_prev, const pauli_op* O_cur,
                            double b_prev, const pauli_trunc* t, pauli_op* O_next,
                            double* b_out, pauli_ws* ws, void* stream) {
  if (!O_cur) return PAULI_EINVAL;
  return lanczos_step(H0, O_prev, O_cur, b_prev, t, O_cur->n_qubits, O_next, b_out, ws, stream);
}

int pauli_rk4_step(const pauli_op* H, const pauli_op* O, double dt, const pauli_trunc* t,
                   pauli_op* out, pauli_ws* ws, void* stream) {
  if (!ws || check_op(H, false) || check_op(O, false) || check_op(out, true)) return PAULI_EINVAL;
  if (H->dtype != PAULI_C128 || O->dtype != PAULI_C128 || out->dtype != PAULI_C128)
    return PAULI_EINVAL;
  if (H->n_qubits != O->n_qubits || out->n_qubits != O->n_qubits) return PAULI_EINVAL;
  Arena ar = make_arena(ws);
  const int W = words_of(O->n_qubits);
  const double h2 = dt / 2.0, c1 = dt / 6.0, c2 = dt / 3.0;
  const OpV Ov = view(O);
  // k = i [H, S], kept at the top of the workspace.  Every use of k below
  // (the stage inputs and the final sum) is truncated with t's length cap
  // first, and the cap acts on each string alone, so strings of k above it
  // are not emitted at all: every result equals the one from the full k.
  pauli_trunc tl;
  memset(&tl, 0, sizeof(tl));
  if (t) tl.max_len = t->max_len;
  auto comm_i = [&](const OpV& S, OpV* k) -> int {
    Call c;
    c.W = W;
    c.has_comm = true;
    c.H = view(H);
    c.O = S;
    c.n_groups = 1;
    c.groups[0].kind = G_SUM;
    c.groups[0].alpha = make_double2(0.0, 1.0);
    c.trunc = tl.max_len > 0 ? &tl : nullptr;
    c.out.to_arena = true;
    int rc = run_call(ar, ws, stream, c);
    *k = c.out.arena_op;
    return rc;
  };
  // S = trunc(O + h k)
  auto stage = [&](const OpV& k, double h, OpV* S) -> int {
    Call c;
    c.W = W;
    c.n_terms = 2;
    c.T[0] = Ov;
    c.T[1] = k;
    c.tgroup[0] = 0;
    c.tgroup[1] = 1;
    c.n_groups = 2;
    c.groups[1].alpha = make_double2(h, 0.0);
    c.trunc = t;
    c.out.to_arena = true;
    int rc = run_call(ar, ws, stream, c);
    *S = c.out.arena_op;
    return rc;
  };
  OpV k1, k2, k3, k4, S2, S3, S4;
  TRY(comm_i(Ov, &k1));
  TRY(stage(k1, h2, &S2));
  TRY(comm_i(S2, &k2));
  TRY(stage(k2, h2, &S3));
  TRY(comm_i(S3, &k3));
  TRY(stage(k3, dt, &S4));
  TRY(comm_i(S4, &k4));
  Call c;
  c.W = W;
  c.n_terms = 5;
  c.T[0] = Ov;
  c.T[1] = k1;
  c.T[2] = k2;
  c.T[3] = k3;
  c.T[4] = k4;
  const double al[5] = {1.0, c1, c2, c2, c1};
  for (int g = 0; g < 5; g++) {
    c.tgroup[g] = g;
    c.groups[g].alpha = make_double2(al[g], 0.0);
  }
  c.n_groups = 5;
  c.trunc = t;
  c.out.user = out;
  return run_call(ar, ws, stream, c);
}

int pauli_add_noise(pauli_op* A, double lambda, void* stream_) {
  if (check_op(A, false) || !(lambda >= 0.0)) return PAULI_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  if (A->size == 0) return PAULI_OK;
  NoiseTable t;
  for (int w = 0; w < NOISE_TABLE; w++) t.f[w] = std::exp(-lambda * (double)w);
  const int W = words_of(A->n_qubits);
  const int blocks = (int)std::min<int64_t>((A->size + 255) / 256, 8192);
  const int f32 = A->dtype == PAULI_C64K ? 1 : 0;
  if (W == 1)
    LAUNCH("k_add_noise", k_add_noise<1>, blocks, 256, A->x, A->z, A->capacity, A->size,
           A->coef, f32, t);
  else
    LAUNCH("k_add_noise", k_add_noise<2>, blocks, 256, A->x, A->z, A->capacity, A->size,
           A->coef, f32, t);
  return PAULI_OK;
}

int pauli_dagger(pauli_op* A, void* stream_) {
  if (check_op(A, false)) return PAULI_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  if (A->size == 0) return PAULI_OK;
  const int blocks = (int)std::min<int64_t>((A->size + 255) / 256, 8192);
  LAUNCH("k_conj", k_conj, blocks, 256, A->coef, A->size, A->dtype == PAULI_C64K ? 1 : 0);
  return PAULI_OK;
}

int pauli_coefficients(const pauli_op* A, const pauli_op* Q, double* out, pauli_ws* ws,
                       void* stream_) {
  if (!ws || check_op(A, false) || check_op(Q, false) || (Q->size && !out)) return PAULI_EINVAL;
  if (A->n_qubits != Q->n_qubits) return PAULI_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  if (Q->size == 0) return PAULI_OK;
  const int W = words_of(A->n_qubits);
  Arena ar = make_arena(ws);
  void* keys = ar.take((size_t)std::max<int64_t>(A->size, 1) * 16 * W);
  double2* res = (double2*)ar.take((size_t)Q->size * 16);
  if (ar.short_) return ws_short(ar, ws);
  const int64_t ba = (std::max<int64_t>(A->size, 1) + 255) / 256, bq = (Q->size + 255) / 256;
  const int af32 = A->dtype == PAULI_C64K ? 1 : 0;
  if (W == 1) {
    if (A->size)
      LAUNCH("k_order_keys", k_order_keys<1>, ba, 256, A->x, A->z, A->capacity, A->size,
             reinterpret_cast<Key<1>*>(keys));
    LAUNCH("k_lookup", k_lookup<1>, bq, 256, reinterpret_cast<const Key<1>*>(keys), A->coef,
           af32, A->size, Q->x, Q->z, Q->capacity, Q->size, res);
  } else {
    if (A->size)
      LAUNCH("k_order_keys", k_order_keys<2>, ba, 256, A->x, A->z, A->capacity, A->size,
             reinterpret_cast<Key<2>*>(keys));
    LAUNCH("k_lookup", k_lookup<2>, bq, 256, reinterpret_cast<const Key<2>*>(keys), A->coef,
           af32, A->size, Q->x, Q->z, Q->capacity, Q->size, res);
  }
  HIP_TRY(hipMemcpyAsync(out, res, (size_t)Q->size * 16, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  g_prof.resolve();
  return PAULI_OK;
}

int pauli_order_keys(const pauli_op* A, uint64_t* keys, void* stream_) {
  if (!keys || check_op(A, false)) return PAULI_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  const int64_t n = A->size;
  if (n == 0) return PAULI_OK;
  const int W = words_of(A->n_qubits);
  const int64_t blocks = (n + 255) / 256;
  if (W == 1)
    LAUNCH("k_order_keys", k_order_keys<1>, blocks, 256, A->x, A->z, A->capacity, n,
           reinterpret_cast<Key<1>*>(keys));
  else
    LAUNCH("k_order_keys", k_order_keys<2>, blocks, 256, A->x, A->z, A->capacity, n,
           reinterpret_cast<Key<2>*>(keys));
  HIP_TRY(hipStreamSynchronize(stream));
  g_prof.resolve();
  return PAULI_OK;
}

int pauli_strings_from_order_keys(int32_t n_qubits, const uint64_t* keys, int64_t n, uint64_t* x,
                                  uint64_t* z, int64_t cap, void* stream_) {
  if (n_qubits < 1 || n_qubits > 128 || n < 0 || cap < n || (n && (!keys || !x || !z)))
    return PAULI_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  if (n == 0) return PAULI_OK;
  const int W = words_of(n_qubits);
  const int64_t blocks = (n + 255) / 256;
  if (W == 1)
    LAUNCH("k_from_order_keys", k_from_order_keys<1>, blocks, 256,
           reinterpret_cast<const Key<1>*>(keys), n, x, z, cap);
  else
    LAUNCH("k_from_order_keys", k_from_order_keys<2>, blocks, 256,
           reinterpret_cast<const Key<2>*>(keys), n, x, z, cap);
  HIP_TRY(hipStreamSynchronize(stream));
  g_prof.resolve();
  return PAULI_OK;
}

int pauli_workspace_query(int op, const pauli_op* A, const pauli_op* B, const pauli_op* C,
                          const pauli_trunc* t, size_t* ws_bytes, int64_t* out_capacity_upper) {
  return workspace_query(op, A, B, C, t, ws_bytes, out_capacity_upper);
}

int pauli_correlator(const pauli_op* O0, const pauli_op* O, double out[2], pauli_ws* ws,
                     void* stream) {
  if (!out || check_op(O0, false) || check_op(O, false)) return PAULI_EINVAL;
  double n0 = 0.0, ip[2] = {0.0, 0.0};
  TRY(pauli_norm2(O0, &n0, ws, stream));
  // <O, O0> looped over O with order-key lookups in O0, then conjugated
  TRY(pauli_inner(O, O0, ip, ws, stream));
  if (!(n0 > 0.0)) return PAULI_EINVAL;
  out[0] = ip[0] / n0;
  out[1] = -ip[1] / n0;
  return PAULI_OK;
}

int pauli_norm2(const pauli_op* A, double* out, pauli_ws* ws, void* stream_) {
  if (!ws || !out || check_op(A, false)) return PAULI_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  Arena ar = make_arena(ws);
  const int blocks = (int)std::min<int64_t>(std::max<int64_t>((A->size + 255) / 256, 1), 1024);
  double2* part = (double2*)ar.take((size_t)blocks * 16);
  double* res = (double*)ar.take(16);
  if (ar.short_) return ws_short(ar, ws);
  if (A->size == 0) {
    *out = 0.0;
    return PAULI_OK;
  }
  if (A->dtype == PAULI_C64K)
    LAUNCH("k_norm_part", k_norm_part<true>, blocks, 256, A->coef, A->size, part);
  else
    LAUNCH("k_norm_part", k_norm_part<false>, blocks, 256, A->coef, A->size, part);
  LAUNCH("k_reduce_dd", k_reduce_dd, 1, 1024, part, (uint32_t)blocks, res);
  double h[2];
  HIP_TRY(hipMemcpyAsync(h, res, 16, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  g_prof.resolve();
  *out = h[0];
  return PAULI_OK;
}

int pauli_inner(const pauli_op* A, const pauli_op* B, double out[2], pauli_ws* ws,
                void* stream_) {
  if (!ws || !out || check_op(A, false) || check_op(B, false)) return PAULI_EINVAL;
  if (A->n_qubits != B->n_qubits) return PAULI_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  Arena ar = make_arena(ws);
  const int W = words_of(A->n_qubits);
  const int blocks = (int)std::min<int64_t>(std::max<int64_t>((A->size + 255) / 256, 1), 1024);
  Ctl* dctl = (Ctl*)ar.take(sizeof(Ctl));
  void* bmk = ar.take((size_t)std::max<int64_t>(B->size, 1) * 16 * W);
  double2* pr = (double2*)ar.take((size_t)blocks * 16);
  double2* pi = (double2*)ar.take((size_t)blocks * 16);
  double* res = (double*)ar.take(32);
  if (ar.short_) return ws_short(ar, ws);
  out[0] = out[1] = 0.0;
  if (A->size == 0 || B->size == 0) return PAULI_OK;
  {
    const size_t words = sizeof(Ctl) / 4;
    LAUNCH("k_fill_u32", k_fill_u32, (words + 255) / 256, 256, (uint32_t*)dctl, 0u, words);
  }
  if (W == 1) {
    LAUNCH("k_mix_keys", k_mix_keys<1>, (B->size + 255) / 256, 256, B->x, B->z, B->capacity,
           B->size, (Key<1>*)bmk, &dctl->bad_keep);
    LAUNCH("k_inner_part", k_inner_part<1>, blocks, 256, A->x, A->z, A->capacity, A->size,
           A->coef, A->dtype == PAULI_C64K, (const Key<1>*)bmk, B->size, B->coef,
           B->dtype == PAULI_C64K, pr, pi);
  } else {
    LAUNCH("k_mix_keys", k_mix_keys<2>, (B->size + 255) / 256, 256, B->x, B->z, B->capacity,
           B->size, (Key<2>*)bmk, &dctl->bad_keep);
    LAUNCH("k_inner_part", k_inner_part<2>, blocks, 256, A->x, A->z, A->capacity, A->size,
           A->coef, A->dtype == PAULI_C64K, (const Key<2>*)bmk, B->size, B->coef,
           B->dtype == PAULI_C64K, pr, pi);
  }
  LAUNCH("k_reduce_dd", k_reduce_dd, 1, 1024, pr, (uint32_t)blocks, res);
  LAUNCH("k_reduce_dd", k_reduce_dd, 1, 1024, pi, (uint32_t)blocks, res + 2);
  double h[4];
  unsigned int bad = 0;
  HIP_TRY(hipMemcpyAsync(h, res, 32, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&bad, &dctl->bad_keep, 4, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  g_prof.resolve();
  if (bad) return PAULI_EINVAL;
  out[0] = h[0];
  out[1] = h[2];
  return PAULI_OK;
}


// ---------------------------------------------------------------------------
// b_n continuation network
// ---------------------------------------------------------------------------
int64_t pauli_mlp_num_params(void) { return mlp::NPARAM; }

static int mlp_check(const pauli_mlp* net) {
  if (!net || net->n_in != mlp::NIN || net->n_hidden != mlp::NHID || net->n_out != mlp::NOUT)
    return PAULI_EINVAL;
  if (!net->params || !net->params_bf16) return PAULI_EINVAL;
  return PAULI_OK;
}

static int gemm_launch(hipStream_t stream, const uint16_t* A, int lda, int transA,
                       const uint16_t* B, int ldb, int transB, float* C, uint16_t* Cb, int ldc,
                       const float* bias, int M, int N, int K, int epilogue) {
  if (M <= 0 || N <= 0 || K <= 0 || M % 16 || N % 16) return PAULI_EINVAL;
  mlp::GemmArgs g;
  g.A = A;
  g.B = B;
  g.C = C;
  g.Cb = Cb;
  g.bias = bias;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.transA = transA;
  g.transB = transB;
  g.M = M;
  g.N = N;
  g.K = K;
  g.epilogue = epilogue;
  LAUNCH("k_gemm_bf16", mlp::k_gemm_bf16, dim3((N + 31) / 32, (M + 31) / 32), 256, g);
  return PAULI_OK;
}

int pauli_gemm_bf16(const uint16_t* A, int lda, int transA, const uint16_t* B, int ldb, int transB,
                    float* C, int ldc, int M, int N, int K, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!A || !B || !C) return PAULI_EINVAL;
  TRY(gemm_launch(stream, A, lda, transA, B, ldb, transB, C, nullptr, ldc, nullptr, M, N, K,
                  mlp::EP_STORE));
  HIP_TRY(hipStreamSynchronize(stream));
  g_prof.resolve();
  return PAULI_OK;
}

int pauli_mlp_sync(const pauli_mlp* net, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  TRY(mlp_check(net));
  LAUNCH("k_to_bf16", mlp::k_to_bf16, (mlp::NPARAM + 255) / 256, 256, net->params,
         net->params_bf16, mlp::NPARAM);
  HIP_TRY(hipStreamSynchronize(stream));
  return PAULI_OK;
}

namespace {
struct MlpBufs {
  uint16_t *xb, *y1b, *y2b, *dyb, *dz2b, *dz1b;
  float *z1, *z2, *yh, *dy, *dy2, *dz2, *dy1, *dz1;
  double *row_err, *row_cnt, *loss;
};
int mlp_bufs(Arena& ar, int64_t B, MlpBufs& m) {
  const size_t b = (size_t)B;
  m.xb = (uint16_t*)ar.take(b * 16 * 2);
  m.y1b = (uint16_t*)ar.take(b * 256 * 2);
  m.y2b = (uint16_t*)ar.take(b * 256 * 2);
  m.dyb = (uint16_t*)ar.take(b * 16 * 2);
  m.dz2b = (uint16_t*)ar.take(b * 256 * 2);
  m.dz1b = (uint16_t*)ar.take(b * 256 * 2);
  m.z1 = (float*)ar.take(b * 256 * 4);
  m.z2 = (float*)ar.take(b * 256 * 4);
  m.yh = (float*)ar.take(b * 16 * 4);
  m.dy = (float*)ar.take(b * 16 * 4);
  m.dy2 = (float*)ar.take(b * 256 * 4);
  m.dz2 = (float*)ar.take(b * 256 * 4);
  m.dy1 = (float*)ar.take(b * 256 * 4);
  m.dz1 = (float*)ar.take(b * 256 * 4);
  m.row_err = (double*)ar.take(b * 8);
  m.row_cnt = (double*)ar.take(b * 8);
  m.loss = (double*)ar.take(16);
  return ar.short_ ? PAULI_EWORKSPACE : PAULI_OK;
}

// forward pass into the buffers
int mlp_forward_bufs(hipStream_t stream, const pauli_mlp* net, const float* x, int64_t B,
                     MlpBufs& m) {
  using namespace mlp;
  const uint16_t* P = net->params_bf16;
  const float* Pf = net->params;
  LAUNCH("k_to_bf16", k_to_bf16, (B * NIN + 255) / 256, 256, x, m.xb, B * NIN);
  // Z1 = X W1^T + b1, Y1 = GELU(Z1)
  TRY(gemm_launch(stream, m.xb, NIN, 0, P + OFF_W1, NIN, 1, m.z1, m.y1b, NHID, Pf + OFF_B1,
                  (int)B, NHID, NIN, EP_BIAS_GELU));
  TRY(gemm_launch(stream, m.y1b, NHID, 0, P + OFF_W2, NHID, 1, m.z2, m.y2b, NHID, Pf + OFF_B2,
                  (int)B, NHID, NHID, EP_BIAS_GELU));
  TRY(gemm_launch(stream, m.y2b, NHID, 0, P + OFF_W3, NHID, 1, m.yh, nullptr, NOUT, Pf + OFF_B3,
                  (int)B, NOUT, NHID, EP_BIAS));
  return PAULI_OK;
}
}  // namespace

int pauli_mlp_forward(const pauli_mlp* net, const float* x, int64_t B, float* y, pauli_ws* ws,
                      void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!ws || !x || !y || B <= 0 || B % 32) return PAULI_EINVAL;
  TRY(mlp_check(net));
  Arena ar = make_arena(ws);
  MlpBufs m;
  if (mlp_bufs(ar, B, m) != PAULI_OK) return ws_short(ar, ws);
  TRY(mlp_forward_bufs(stream, net, x, B, m));
  HIP_TRY(hipMemcpyAsync(y, m.yh, (size_t)B * mlp::NOUT * 4, hipMemcpyDeviceToDevice, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  g_prof.resolve();
  return PAULI_OK;
}

int pauli_mlp_loss_grad(const pauli_mlp* net, const float* x, const float* t, const float* mask,
                        int64_t B, double* loss, float* acts, pauli_ws* ws, void* stream_) {
  using namespace mlp;
  hipStream_t stream = (hipStream_t)stream_;
  if (!ws || !x || !t || !mask || B <= 0 || B % 32) return PAULI_EINVAL;
  TRY(mlp_check(net));
  if (!net->grads) return PAULI_EINVAL;
  Arena ar = make_arena(ws);
  MlpBufs m;
  if (mlp_bufs(ar, B, m) != PAULI_OK) return ws_short(ar, ws);
  TRY(mlp_forward_bufs(stream, net, x, B, m));
  const uint16_t* P = net->params_bf16;
  float* G = net->grads;
  const int64_t nb = (B + 255) / 256;
  LAUNCH("k_mse_rows", k_mse_rows, nb, 256, m.yh, t, mask, B, m.row_err, m.row_cnt);
  LAUNCH("k_sum_rows", k_sum_rows, 1, 256, m.row_err, m.row_cnt, B, m.loss);
  LAUNCH("k_mse_grad", k_mse_grad, (B * NOUT + 255) / 256, 256, m.yh, t, mask, B * NOUT, m.loss,
         m.dy, m.dyb);
  // layer 3: dW3[16][256] = dY^T Y2, db3 = column sums of dY, dY2 = dY W3
  TRY(gemm_launch(stream, m.dyb, NOUT, 1, m.y2b, NHID, 0, G + OFF_W3, nullptr, NHID, nullptr,
                  NOUT, NHID, (int)B, EP_STORE));
  LAUNCH("k_col_sum", k_col_sum, 1, 256, m.dy, B, NOUT, G + OFF_B3);
  TRY(gemm_launch(stream, m.dyb, NOUT, 0, P + OFF_W3, NHID, 0, m.dy2, nullptr, NHID, nullptr,
                  (int)B, NHID, NOUT, EP_STORE));
  LAUNCH("k_gelu_back", k_gelu_back, (B * NHID + 255) / 256, 256, m.dy2, m.z2, B * NHID, m.dz2,
         m.dz2b);
  // layer 2
  TRY(gemm_launch(stream, m.dz2b, NHID, 1, m.y1b, NHID, 0, G + OFF_W2, nullptr, NHID, nullptr,
                  NHID, NHID, (int)B, EP_STORE));
  LAUNCH("k_col_sum", k_col_sum, 1, 256, m.dz2, B, NHID, G + OFF_B2);
  TRY(gemm_launch(stream, m.dz2b, NHID, 0, P + OFF_W2, NHID, 0, m.dy1, nullptr, NHID, nullptr,
                  (int)B, NHID, NHID, EP_STORE));
  LAUNCH("k_gelu_back", k_gelu_back, (B * NHID + 255) / 256, 256, m.dy1, m.z1, B * NHID, m.dz1,
         m.dz1b);
  // layer 1
  TRY(gemm_launch(stream, m.dz1b, NHID, 1, m.xb, NIN, 0, G + OFF_W1, nullptr, NIN, nullptr, NHID,
                  NIN, (int)B, EP_STORE));
  LAUNCH("k_col_sum", k_col_sum, 1, 256, m.dz1, B, NHID, G + OFF_B1);
  if (acts) {
    float* o = acts;
    auto bf = [&](const uint16_t* src, int64_t n) -> int {
      LAUNCH("k_bf_to_f", k_bf_to_f, (n + 255) / 256, 256, src, o, n);
      o += n;
      return PAULI_OK;
    };
    auto fc = [&](const float* src, int64_t n) -> int {
      HIP_TRY(hipMemcpyAsync(o, src, (size_t)n * 4, hipMemcpyDeviceToDevice, stream));
      o += n;
      return PAULI_OK;
    };
    TRY(bf(m.xb, B * NIN));
    TRY(fc(m.z1, B * NHID));
    TRY(bf(m.y1b, B * NHID));
    TRY(fc(m.z2, B * NHID));
    TRY(bf(m.y2b, B * NHID));
    TRY(fc(m.yh, B * NOUT));
    TRY(bf(m.dyb, B * NOUT));
    TRY(fc(m.dy2, B * NHID));
    TRY(bf(m.dz2b, B * NHID));
    TRY(fc(m.dy1, B * NHID));
    TRY(bf(m.dz1b, B * NHID));
  }
  double h[2];
  HIP_TRY(hipMemcpyAsync(h, m.loss, 16, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  g_prof.resolve();
  if (loss) *loss = h[0];
  return PAULI_OK;
}

int pauli_mlp_train(const pauli_mlp* net, const float* x, const float* t, const float* mask,
                    int64_t n, const int32_t* order, int64_t epochs, int32_t batch, double lr,
                    double b1, double b2, double eps, int64_t t0, double* losses, pauli_ws* ws,
                    void* stream_) {
  using namespace mlp;
  hipStream_t stream = (hipStream_t)stream_;
  TRY(mlp_check(net));
  if (!ws || !x || !t || !mask || !order || !losses || n <= 0 || epochs < 0 || batch <= 0 ||
      batch > 4096 || t0 < 0 || !net->grads || !net->adam_m || !net->adam_v)
    return PAULI_EINVAL;
  Arena ar = make_arena(ws);
  const int nblk_max = (batch + SR - 1) / SR;
  float* part = (float*)ar.take((size_t)nblk_max * NPARAM * 4);
  double* lpart = (double*)ar.take((size_t)nblk_max * 16);
  if (ar.short_) return ws_short(ar, ws);
  const int64_t spe = (n + batch - 1) / batch;  // minibatches per epoch
  int64_t step = t0;
  for (int64_t e = 0; e < epochs; e++) {
    for (int64_t k = 0; k < spe; k++) {
      const int64_t s0 = k * batch;
      const int rows = (int)std::min<int64_t>(batch, n - s0);
      const int nblk = (rows + SR - 1) / SR;
      StepArgs sa;
      sa.params = net->params;
      sa.pb = net->params_bf16;
      sa.X = x;
      sa.T = t;
      sa.Mk = mask;
      sa.order = order + e * n + s0;
      sa.rows = rows;
      sa.part = part;
      sa.lpart = lpart;
      LAUNCH("k_mlp_step", k_mlp_step, nblk, 256, sa);
      step++;
      const float c1 = (float)(1.0 - std::pow(b1, (double)step));
      const float c2 = (float)(1.0 - std::pow(b2, (double)step));
      LAUNCH("k_mlp_reduce_adam", k_mlp_reduce_adam, (NPARAM + 255) / 256, 256, part, nblk,
             net->grads, net->params, net->adam_m, net->adam_v, net->params_bf16, (float)lr,
             (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), (float)eps, c1, c2,
             lpart, losses + e * spe + k);
    }
  }
  HIP_TRY(hipStreamSynchronize(stream));
  g_prof.resolve();
  return PAULI_OK;
}

int pauli_mlp_adam(const pauli_mlp* net, double lr, double b1, double b2, double eps, int64_t t,
                   void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  TRY(mlp_check(net));
  if (!net->grads || !net->adam_m || !net->adam_v || t < 1) return PAULI_EINVAL;
  const float c1 = (float)(1.0 - std::pow(b1, (double)t));
  const float c2 = (float)(1.0 - std::pow(b2, (double)t));
  LAUNCH("k_adam", mlp::k_adam, (mlp::NPARAM + 255) / 256, 256, net->params, net->grads,
         net->adam_m, net->adam_v, net->params_bf16, mlp::NPARAM, (float)lr, (float)b1,
         (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), (float)eps, c1, c2);
  HIP_TRY(hipStreamSynchronize(stream));
  g_prof.resolve();
  return PAULI_OK;
}

}  // extern "C"
