// HIP kernels of the Pauli-string engine (gfx950, wave64).
//
// Data flow of one engine call (commutator, linear combination, truncation,
// canonicalisation all use it):
//   k_emit<COUNT>   pair loop over (H string, O string) -> for every
//                   anticommuting pair the product string's mixed key picks a
//                   hash bin; per-workgroup bin histograms (LDS) -> counts
//                   matrix [rows][NBINS]; operator terms are binned the same way
//   k_scan_cols / k_scan_bins
//                   column prefix of the counts matrix, bin bases, bucket sizes
//   k_emit<SCATTER> the same pair loop, writing records (mixed key, value,
//                   source id) at their bin's cursor
//   k_merge         one workgroup per bucket of bins: records -> LDS, counting
//                   sort on the next 11 key bits + insertion sort per thread
//                   range, then every run of equal keys is folded in ascending
//                   source id (the canonical summation order), filtered, and
//                   written compactly; level-0 histogram of |c|^2 for top-M
//   k_select / k_level1 / k_cand_level / k_finish / k_count_boundary
//                   exact radix select of the M-th largest (|c|^2, key) pair
//   k_scan_buckets / k_write
//                   bucket output bases, stable compaction into the caller's
//                   word-major output
#pragma once
#include <type_traits>

#include "device_common.hpp"

namespace pauli {

enum GroupKind : int { G_TERM = 0, G_SUM = 1, G_SUM_KAHAN32 = 2 };
enum AlphaKind : int { A_GENERAL = 0, A_ONE = 1, A_I = 2, A_DIV = 3 };  // A_DIV: v / alpha.x
enum MergeMode : int { M_PLAIN = 0, M_LANCZOS = 1 };
constexpr int MAX_GROUPS = 8;
constexpr int MAX_TERMS = 6;

struct Ctl {
  unsigned long long pe_total;   // records emitted in this pass
  unsigned int maxg[8];          // max records over aligned groups of 2^k bins
  unsigned int overflow;         // a bucket exceeded MERGE_CAP / u32 overflow
  unsigned int bad_keep;         // keep set not canonical
  unsigned long long u_slots;    // U slots written by the merges
  unsigned long long u_unique;   // distinct strings with nonzero merged value
  unsigned long long surv_total; // survivors after filters (incl. keep)
  unsigned long long keep_total; // keep-set survivors
  unsigned long long cand_n[3];  // candidate list sizes
  unsigned long long sel_K;      // records still needed inside the chosen bin
  unsigned long long sel_count;  // records in the chosen bin
  unsigned int sel_digit;
  unsigned int t_found;
  unsigned long long T[8];       // threshold composite (m2 bits, ~key words)
  unsigned long long out_total;
  double norm_hi, norm_lo;
  double inner[4];
  int sel_mode;                  // SelMode chosen on the device
  unsigned int fin_level;        // 0: finish on the level-1 list, 1: after digit 1
  unsigned int deep;             // the device select stopped: the host finishes it
  unsigned int sel_d0, sel_d1;   // threshold digits 0 and 1
  unsigned long long part_total; // records in all partitions (several-pass calls)
  unsigned int ndefer;           // buckets deferred to the full-size merge (this pass)
  unsigned int unsorted;         // a term of a direct merge is not in canonical order
  unsigned int spec_fail;        // a scatter launched before the count was read stands down
};

struct EmitArgs {
  // commutator group: H packed [nH][2W] raw words in ascending order of their
  // lowest site (k_prep_h), with each entry's index in the caller's H and the
  // first entry whose lowest site is >= s (hstart[s], s = 0 .. 64W + 1);
  // O word-major
  const uint64_t* Hk;
  const uint32_t* Hidx;
  const uint32_t* hstart;
  const int* hspan;    // largest highest-minus-lowest site over H (device)
  const double2* Hc;
  int nH;
  int has_comm;
  int product;  // plain product A B (every pair, i^e h_a c_b) instead of [A, B]
  int ts_n;     // > 0: translation-symmetric operators on ts_n periodic sites; every
                // emitted string is replaced by its orbit representative
  int comm_rows;
  uint32_t comm_group;
  const uint64_t* Ox;
  const uint64_t* Oz;
  int64_t Ocap;
  int64_t nO;
  const void* Oc;
  // operator terms
  int n_terms;
  int term_rows;
  const uint64_t* tx[MAX_TERMS];
  const uint64_t* tz[MAX_TERMS];
  int64_t tcap[MAX_TERMS];
  const void* tc[MAX_TERMS];
  int tf32[MAX_TERMS];
  uint32_t tgroup[MAX_TERMS];
  int tlist[MAX_TERMS];
  int64_t tstart[MAX_TERMS + 1];
  // strings longer than this are not emitted (plain mode; 0: no cap): the
  // length cap depends on the key alone, so it can act before the merge
  int max_len;
  // partition mode: the bin is the top pass_bits bits of the order key
  // (2^pass_bits partitions); records are written as the binning of a pass
  // will store them (source id in the top part_F bits of the key), the top
  // 32 bits of the order key go to ptop, and the source ids to psrc when they
  // are kept aside (wide)
  int part;
  int part_F;
  uint32_t* ptop;
  uint32_t* psrc;
  // binning
  int pass_bits;
  uint32_t pass_id;
  uint32_t* counts;
  const uint32_t* bin_base;
  void* recs;          // Rec<W, F32>[records]
  uint32_t* rsrc_wide; // source ids when they do not fit the folded bits
  int wide;
  const unsigned int* skip;  // scatter: nothing to do when *skip != 0 (nullable)
};

template <bool F32>
using RecV = typename std::conditional<F32, float2, double2>::type;

// One emitted record: the mixed key and the value.  The leading
// NBINS_LOG + pass_bits bits of the key are implied by the record's bin and
// pass, so they carry the source id instead: group in the top 3 bits, then
// the index inside the group (H index; 0 for operator terms).  Calls whose
// ids do not fit (canonicalisation of long lists) keep them in a side array.
// FP64 records of two-word keys (48 bytes) are padded to 64: the pass binning
// of the N = 128 precision-split step took 7 % less time.  Padding the FP32
// records (24 -> 32 and 40 -> 64 bytes) made their calls 3-6 % slower.
template <int W, bool F32>
constexpr int rec_pad_words() {
  return F32 ? 0 : (int)((32 - (sizeof(Key<W>) + sizeof(RecV<F32>)) % 32) % 32 / 8);
}
template <int W, bool F32, int PAD = rec_pad_words<W, F32>()>
struct Rec {
  Key<W> k;
  RecV<F32> v;
  uint64_t pad[PAD];  // written as zeros
};
template <int W, bool F32>
struct Rec<W, F32, 0> {
  Key<W> k;
  RecV<F32> v;
};
template <int W, bool F32>
DEV Rec<W, F32> make_rec(const Key<W>& k, RecV<F32> v) {
  Rec<W, F32> r;
  r.k = k;
  r.v = v;
  if constexpr (rec_pad_words<W, F32>() > 0)
#pragma unroll
    for (int i = 0; i < rec_pad_words<W, F32>(); i++) r.pad[i] = 0ull;
  return r;
}

// Row of the count matrix (and so the place of a workgroup's records inside
// every bin) for workgroup b of a grid of n: workgroups go to the eight XCDs
// round robin (b mod 8), so this numbering gives each XCD a contiguous range
// of rows.  Its partial cache lines in a bin then fill up inside its own L2
// instead of reaching memory as separate partial writes.
__device__ __forceinline__ uint32_t layout_row(uint32_t b, uint32_t n) {
  const uint32_t n8 = n & ~7u;
  return b < n8 ? (b & 7u) * (n8 >> 3) + (b >> 3) : b;
}

template <int W, bool F32, bool SCATTER, int NBL>
// Eight waves per SIMD (two workgroups per CU) where registers and LDS allow;
// two-word strings need more than 64 registers per lane in the pair loop and
// 2^15 bins fill the LDS of a CU, so those aim at four.
__global__ __launch_bounds__(EMIT_THREADS)
__attribute__((amdgpu_waves_per_eu(W == 1 && NBL <= 14 ? 8 : 4))) void k_emit(EmitArgs a) {
  constexpr int NB = 1 << NBL;  // hash bins of this call
  using V = RecV<F32>;
  __shared__ uint32_t hist[NB];
  __shared__ uint32_t queue[EMIT_THREADS / 64][128];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int row = blockIdx.x;
  const uint32_t lrow = layout_row(blockIdx.x, gridDim.x);
  if (SCATTER && a.skip && *a.skip) return;
  if (SCATTER) {
    const uint32_t* crow = a.counts + (size_t)lrow * NB;
    for (int i = tid; i < NB; i += EMIT_THREADS) hist[i] = a.bin_base[i] + crow[i];
  } else {
    for (int i = tid; i < NB; i += EMIT_THREADS) hist[i] = 0u;
  }
  __syncthreads();
  Rec<W, F32>* recs = reinterpret_cast<Rec<W, F32>*>(a.recs);
  const int F = NBL + a.pass_bits;

  auto deposit = [&](const Key<W>& raw, V val, uint32_t group, uint32_t index) {
    if (a.max_len > 0 && key_length<W>(raw) > a.max_len) return;
    Key<W> mk = mix_key<W>(raw);
    if (a.part) {
      const uint32_t pid = (uint32_t)(mk.w[0] >> (64 - a.pass_bits));
      const uint32_t pos = atomicAdd(&hist[pid], 1u);
      if (SCATTER) {
        const int PF = a.part_F;
        a.ptop[pos] = (uint32_t)(mk.w[0] >> 32);
        const uint64_t small = a.wide ? 0ull : (((uint64_t)group << (PF - 3)) | index);
        mk.w[0] = (small << (64 - PF)) | (mk.w[0] & (~0ull >> PF));
        recs[pos] = make_rec<W, F32>(mk, val);
        if (a.wide) a.psrc[pos] = (group << GROUP_SHIFT) | index;
      }
      return;
    }
    uint64_t top = mk.w[0];
    if (a.pass_bits) {
      if ((uint32_t)(top >> (64 - a.pass_bits)) != a.pass_id) return;
      top <<= a.pass_bits;
    }
    const uint32_t bin = (uint32_t)(top >> (64 - NBL));
    const uint32_t pos = atomicAdd(&hist[bin], 1u);
    if (SCATTER) {
      const uint64_t small = a.wide ? 0ull : (((uint64_t)group << (F - 3)) | index);
      mk.w[0] = (small << (64 - F)) | (mk.w[0] & (~0ull >> F));
      recs[pos] = make_rec<W, F32>(mk, val);
      if (a.wide) a.rsrc_wide[pos] = (group << GROUP_SHIFT) | index;
    }
  };

  if (a.has_comm && row < a.comm_rows) {
    // Each tile of EMIT_THREADS strings is put in ascending order of lowest
    // site, so a wave holds strings of nearby support and loops only over the
    // H strings whose sites can overlap its window [wlo, whi].  A pair whose
    // supports do not overlap commutes, so skipping it changes nothing.
    constexpr int SITES = 64 * W;
    __shared__ uint32_t scnt[SITES + 2];
    __shared__ uint16_t sperm[EMIT_THREADS];
    const V* Oc = reinterpret_cast<const V*>(a.Oc);
    const int64_t ntiles = (a.nO + EMIT_THREADS - 1) / EMIT_THREADS;
    for (int64_t tile = row; tile < ntiles; tile += a.comm_rows) {
      // lowest and highest site of this thread's string (empty or padding
      // strings sort last, with site SITES)
      int lo = SITES, hi = -1;
      {
        const int64_t i0 = tile * EMIT_THREADS + tid;
        if (i0 < a.nO) {
#pragma unroll
          for (int w = W - 1; w >= 0; w--) {
            const uint64_t s = a.Ox[(size_t)w * a.Ocap + i0] | a.Oz[(size_t)w * a.Ocap + i0];
            if (s) {
              lo = 64 * w + __builtin_ctzll(s);
              if (hi < 0) hi = 64 * w + 63 - __builtin_clzll(s);
            }
          }
        }
      }
      for (int q = tid; q < SITES + 2; q += EMIT_THREADS) scnt[q] = 0u;
      __syncthreads();
      const uint32_t rk = atomicAdd(&scnt[lo], 1u);
      __syncthreads();
      if (tid < 64) {  // exclusive scan of the SITES + 1 site counts (one wave)
        constexpr int PERL = (SITES + 1 + 63) / 64;
        uint32_t c[PERL], sum = 0;
#pragma unroll
        for (int q = 0; q < PERL; q++) {
          const int sidx = tid * PERL + q;
          c[q] = sidx <= SITES ? scnt[sidx] : 0u;
          sum += c[q];
        }
        uint32_t x = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const uint32_t y = __shfl_up(x, d, 64);
          if (tid >= d) x += y;
        }
        uint32_t pre = x - sum;
#pragma unroll
        for (int q = 0; q < PERL; q++) {
          const int sidx = tid * PERL + q;
          if (sidx <= SITES) scnt[sidx] = pre;
          pre += c[q];
        }
      }
      __syncthreads();
      sperm[scnt[lo] + rk] = (uint16_t)tid;
      __syncthreads();
      const int64_t i = tile * EMIT_THREADS + sperm[tid];
      __syncthreads();  // scnt / sperm are rewritten by the next tile
      const bool valid = i < a.nO;
      uint64_t xb[W], zb[W];
      V cb;
#pragma unroll
      for (int w = 0; w < W; w++) {
        xb[w] = valid ? a.Ox[(size_t)w * a.Ocap + i] : 0ull;
        zb[w] = valid ? a.Oz[(size_t)w * a.Ocap + i] : 0ull;
      }
      if (valid) cb = Oc[i];
      else { cb.x = 0; cb.y = 0; }
      // the wave's site window
      int slo = SITES, shi = -1;
#pragma unroll
      for (int w = W - 1; w >= 0; w--) {
        const uint64_t s = xb[w] | zb[w];
        if (s) {
          slo = 64 * w + __builtin_ctzll(s);
          if (shi < 0) shi = 64 * w + 63 - __builtin_clzll(s);
        }
      }
      int wlo = slo, whi = shi;
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        wlo = min(wlo, __shfl_xor(wlo, d, 64));
        whi = max(whi, __shfl_xor(whi, d, 64));
      }
      // the product keeps every pair (identity strings included); the
      // commutator only pairs that can overlap
      if (whi < 0 && !a.product) continue;  // nothing but empty strings: all commute
      const int hfirst = a.product ? 0 : (int)a.hstart[max(wlo - *a.hspan, 0)];
      const int hend = a.product ? a.nH : (int)a.hstart[whi + 1];

      // Handle one queued (lane, H position) pair per lane.
      auto process = [&](uint32_t entry, bool active) {
        const int src_lane = (int)(entry & 63u);
        const int h = (int)(entry >> 6);
        uint64_t bx[W], bz[W];
#pragma unroll
        for (int w = 0; w < W; w++) {
          bx[w] = __shfl(xb[w], src_lane, 64);
          bz[w] = __shfl(zb[w], src_lane, 64);
        }
        V bc;
        bc.x = __shfl(cb.x, src_lane, 64);
        bc.y = __shfl(cb.y, src_lane, 64);
        if (!active) return;
        const uint64_t* hk = a.Hk + (size_t)h * (2 * W);
        Key<W> c;
        int pa = 0, pb = 0, pz = 0, pc = 0;
#pragma unroll
        for (int w = 0; w < W; w++) {
          const uint64_t ax = hk[w], az = hk[W + w];
          c.w[w] = ax ^ bx[w];
          c.w[W + w] = az ^ bz[w];
          pa += __popcll(ax & az);
          pb += __popcll(bx[w] & bz[w]);
          pz += __popcll(az & bx[w]);
          pc += __popcll(c.w[w] & c.w[W + w]);
        }
        // P_a P_b = i^(pa + pb + 2 pop(z_a & x_b) - pc) P_c; anticommuting
        // pairs contribute 2 i^e h_a c_b to [P_a, P_b] h_a c_b, every pair
        // i^e h_a c_b to the product.
        const int e = (pa + pb + 2 * pz - pc) & 3;
        // translation symmetry: several O strings can meet the same H entry
        // in one orbit; (H entry, rotation) orders their contributions
        const int rot = a.ts_n ? ts_representative<W>(c.w, a.ts_n) : 0;
        const uint32_t horig = a.Hidx[h];
        const double2 hd = a.Hc[horig];
        // FP32 records: the product of the FP64 H coefficient and the stored
        // FP32 coefficient is formed in FP64 and rounded once to FP32
        V prod;
        if constexpr (F32) {
          const double2 pd = cmul(hd, make_double2((double)bc.x, (double)bc.y));
          prod = make_float2((float)pd.x, (float)pd.y);
        } else {
          prod = cmul(hd, bc);
        }
        deposit(c, a.product ? times_ie(prod, e) : times_2ie(prod, e), a.comm_group,
                a.ts_n ? horig * 256u + (uint32_t)rot : horig);
      };

      uint32_t qn = 0;  // wave-uniform queue fill
      for (int h = hfirst; h < hend; ++h) {
        const uint64_t* hk = a.Hk + (size_t)h * (2 * W);
        uint32_t par = 0;
#pragma unroll
        for (int w = 0; w < W; w++) par += __popcll((hk[w] & zb[w]) ^ (hk[W + w] & xb[w]));
        const bool emit = valid && (a.product || (par & 1u));
        const uint64_t m = __ballot(emit);
        if (m) {
          const uint32_t pos = qn + mbcnt64(m);
          if (emit) queue[wv][pos] = (uint32_t)lane | ((uint32_t)h << 6);
          qn += (uint32_t)__popcll(m);
          if (qn >= 64) {
            wave_sync();
            process(queue[wv][lane], true);
            const uint32_t rem = qn - 64;
            const uint32_t mv = (uint32_t)lane < rem ? queue[wv][64 + lane] : 0u;
            wave_sync();
            if ((uint32_t)lane < rem) queue[wv][lane] = mv;
            wave_sync();
            qn = rem;
          }
        }
      }
      if (qn) {
        wave_sync();
        process(queue[wv][lane], (uint32_t)lane < qn);
        wave_sync();
      }
    }
  } else if (a.n_terms > 0) {
    const int trow = row - (a.has_comm ? a.comm_rows : 0);
    const int64_t total = a.tstart[a.n_terms];
    const int64_t ntiles = (total + EMIT_THREADS - 1) / EMIT_THREADS;
    for (int64_t tile = trow; tile < ntiles; tile += a.term_rows) {
      const int64_t v = tile * EMIT_THREADS + tid;
      if (v < total) {
        int t = 0;
        while (t + 1 < a.n_terms && v >= a.tstart[t + 1]) t++;
        const int64_t k = v - a.tstart[t];
        Key<W> raw;
#pragma unroll
        for (int w = 0; w < W; w++) {
          raw.w[w] = a.tx[t][(size_t)w * a.tcap[t] + k];
          raw.w[W + w] = a.tz[t][(size_t)w * a.tcap[t] + k];
        }
        if (a.ts_n) (void)ts_representative<W>(raw.w, a.ts_n);
        V val;
        if (a.tf32[t]) {
          const float2 f = reinterpret_cast<const float2*>(a.tc[t])[k];
          val.x = f.x;
          val.y = f.y;
        } else {
          const double2 d = reinterpret_cast<const double2*>(a.tc[t])[k];
          val.x = d.x;
          val.y = d.y;
        }
        deposit(raw, val, a.tgroup[t], a.tlist[t] ? (uint32_t)k : 0u);
      }
    }
  }
  __syncthreads();
  if (!SCATTER) {
    uint32_t* crow = a.counts + (size_t)lrow * NB;
    for (int i = tid; i < NB; i += EMIT_THREADS) crow[i] = hist[i];
  }
}

// One partition of a several-pass call, binned for the merge: block r of the
// grid takes the r-th contiguous share of partition `part` (records as the
// merge reads them, from the partition-mode emission, and the top 32 bits of
// each order key in ptop), histograms the NBL key bits after the pass bits
// (COUNT: from ptop alone, into row r of the counts matrix) or copies each
// record to its bin cursor (SCATTER), with its source id when it is kept
// aside (wide).
struct SplitArgs {
  const void* precs;
  const uint32_t* ptop;
  const uint32_t* psrc;
  const uint32_t* pbase;  // partition starts [2^pass_bits + 1]
  uint32_t part;
  int pass_bits;
  int wide;
  uint32_t* counts;        // [gridDim.x][2^NBL]
  const uint32_t* bin_base;
  void* recs;
  uint32_t* rsrc_wide;
};

template <int W, bool F32, bool SCATTER, int NBL>
__global__ __launch_bounds__(1024) void k_split(SplitArgs a) {
  constexpr int NB = 1 << NBL;
  __shared__ uint32_t hist[NB];
  const int tid = threadIdx.x;
  // count-matrix row of this block: rows grouped by XCD, as in the emission
  const uint32_t lrow = layout_row(blockIdx.x, gridDim.x);
  const uint32_t* crow = a.counts + (size_t)lrow * NB;
  if (SCATTER)
    for (int i = tid; i < NB; i += 1024) hist[i] = a.bin_base[i] + crow[i];
  else
    for (int i = tid; i < NB; i += 1024) hist[i] = 0u;
  __syncthreads();
  const uint32_t lo = a.pbase[a.part], n = a.pbase[a.part + 1] - lo;
  const uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const uint32_t r0 = lo + min(n, blockIdx.x * chunk);
  const uint32_t r1 = lo + min(n, (blockIdx.x + 1) * chunk);
  // records moved as 64-bit words (word 0 is the key's leading word)
  constexpr int RW = (int)(sizeof(Rec<W, F32>) / 8);
  static_assert(sizeof(Rec<W, F32>) % 8 == 0, "records are whole 64-bit words");
  const uint64_t* in = reinterpret_cast<const uint64_t*>(a.precs);
  uint64_t* out = reinterpret_cast<uint64_t*>(a.recs);
  // SB records per thread and step, all loaded before any is binned, so that
  // each wave keeps SB loads in flight (COUNT: 4 bytes per record)
  constexpr int SB = SCATTER ? 4 : 8;
  for (uint32_t i0 = r0 + tid; i0 < r1; i0 += SB * 1024) {
    uint64_t rw[SCATTER ? SB : 1][RW];
    uint32_t top[SB], src[SB];
#pragma unroll
    for (int u = 0; u < SB; u++) {
      const uint32_t i = i0 + u * 1024;
      if (i < r1) {
        top[u] = a.ptop[i];
        if constexpr (SCATTER) {
#pragma unroll
          for (int q = 0; q < RW; q++) rw[u][q] = in[(size_t)i * RW + q];
          if (a.wide) src[u] = a.psrc[i];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < SB; u++) {
      const uint32_t i = i0 + u * 1024;
      if (i >= r1) break;
      const uint32_t bin = (top[u] << a.pass_bits) >> (32 - NBL);
      const uint32_t pos = atomicAdd(&hist[bin], 1u);
      if constexpr (SCATTER) {
#pragma unroll
        for (int q = 0; q < RW; q++) out[(size_t)pos * RW + q] = rw[u][q];
        if (a.wide) a.rsrc_wide[pos] = src[u];
      }
    }
  }
  if (!SCATTER) {
    __syncthreads();
    uint32_t* w = a.counts + (size_t)lrow * NB;
    for (int i = tid; i < NB; i += 1024) w[i] = hist[i];
  }
}

// Exclusive scan of the partition totals (one block of 1024 threads, at most
// 4096 partitions): pbase[p] for p < np, pbase[p] = total beyond.
__global__ __launch_bounds__(1024) void k_scan_part(const uint32_t* total, int np, uint32_t* pbase,
                                                    int nbase, Ctl* ctl) {
  __shared__ uint32_t scan_tmp[1024 / 64 + 1];
  const int t = threadIdx.x;
  uint32_t v[4], s = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int p = t * 4 + k;
    v[k] = p < np ? total[p] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t pre = block_exclusive_scan(s, scan_tmp, &tot);
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int p = t * 4 + k;
    if (p < np) pbase[p] = pre;
    pre += v[k];
  }
  for (int p = np + t; p < nbase; p += 1024) pbase[p] = tot;
  if (t == 0) ctl->part_total = tot;
}

// Partition prefixes from the first count pass, which binned every record by
// the top NBINS_LOG bits of its order key and left, per bin, the exclusive
// prefix over rows and the total.  A partition (top pass_bits bits) is an
// aligned group of 2^(NBINS_LOG - pass_bits) bins, so its prefixes and total
// are the sums of theirs.  Block r < rows reduces row r into row r of pc
// (ncol columns, those at and above 2^pass_bits zero); block `rows` reduces
// the bin totals and replaces the first 2^pass_bits of them in place (all
// read before any is written).  Each thread sums 16 consecutive bins, then a
// tree in LDS combines the 2^(10 - pass_bits) threads of a partition.
// pass_bits <= 10; the caller guarantees fewer than 2^32 records, so no sum
// wraps.
__global__ __launch_bounds__(1024) void k_part_from_bins(const uint32_t* counts, int rows,
                                                         int pass_bits, int ncol, uint32_t* pc,
                                                         uint32_t* total) {
  static_assert(NBINS == 16 * 1024, "one thread per 16 bins");
  __shared__ uint32_t part[1024];
  const int r = blockIdx.x, t = threadIdx.x;
  const int np = 1 << pass_bits, g = 1024 >> pass_bits;  // threads per partition
  const uint32_t* src = r < rows ? counts + (size_t)r * NBINS : total;
  const uint4* s4 = reinterpret_cast<const uint4*>(src) + 4 * t;
  uint32_t v = 0u;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const uint4 u = s4[q];
    v += u.x + u.y + u.z + u.w;
  }
  part[t] = v;
  __syncthreads();
  for (int d = 1; d < g; d <<= 1) {
    if ((t & (2 * d - 1)) == 0) part[t] += part[t + d];
    __syncthreads();
  }
  if (r < rows) {
    for (int p = t; p < ncol; p += 1024) pc[(size_t)r * ncol + p] = p < np ? part[p * g] : 0u;
  } else if (t < np) {
    total[t] = part[t * g];
  }
}

// Column-wise exclusive prefix of the counts matrix (rows x nbins, row
// major) and the bin totals.  A block of SC_NSEG x SC_COLS threads covers
// SC_COLS columns: thread (segment g, column b) loads rows
// [SC_SEG g, SC_SEG g + SC_SEG) of column b all at once, the segment sums of
// a column are combined in LDS, and each thread writes its rows' prefixes.
// rows <= SC_NSEG * SC_SEG.
constexpr int SC_COLS = 32, SC_SEG = 36, SC_NSEG = 32;
constexpr int SC_ROWS_MAX = SC_SEG * SC_NSEG;
__global__ __launch_bounds__(SC_COLS * SC_NSEG) void k_scan_cols(uint32_t* counts, int rows,
                                                                 uint32_t* bin_total, Ctl* ctl,
                                                                 int nbins) {
  __shared__ unsigned long long ssum[SC_NSEG][SC_COLS];
  const int col = threadIdx.x % SC_COLS, seg = threadIdx.x / SC_COLS;
  const int b = blockIdx.x * SC_COLS + col;
  const int r0 = seg * SC_SEG;
  const bool on = b < nbins;
  uint32_t c[SC_SEG];
#pragma unroll
  for (int q = 0; q < SC_SEG; q++)
    c[q] = (on && r0 + q < rows) ? counts[(size_t)(r0 + q) * nbins + b] : 0u;
  unsigned long long s = 0;
#pragma unroll
  for (int q = 0; q < SC_SEG; q++) s += c[q];
  ssum[seg][col] = s;
  __syncthreads();
  unsigned long long run = 0;
  for (int g = 0; g < seg; g++) run += ssum[g][col];
#pragma unroll
  for (int q = 0; q < SC_SEG; q++) {
    if (on && r0 + q < rows) counts[(size_t)(r0 + q) * nbins + b] = (uint32_t)run;
    run += c[q];
  }
  if (on && seg == SC_NSEG - 1) {  // the last segment's running sum is the column total
    if (run > 0xFFFFFFFFull) atomicOr(&ctl->overflow, 2u);
    bin_total[b] = (uint32_t)run;
  }
}

// Both scans of a count pass over 2^10 bins with at most SMALL_SCAN_ROWS
// emission rows, in block 0: thread t turns column t of the count matrix
// into row prefixes (as k_scan_cols), then the block scans the 1024 bin
// totals into bin bases and takes the largest totals over aligned groups of
// 1, 2, 4, 8, 16 bins (as k_scan_bins).  All blocks of the grid clear a share
// of `zero`.  Such calls hold at most 2^18 records, so no total overflows 32
// bits.
constexpr int SMALL_SCAN_ROWS = 32;
__global__ __launch_bounds__(1024) void k_scan_small(uint32_t* counts, int rows,
                                                     uint32_t* bin_base, Ctl* ctl, uint32_t* zero,
                                                     uint32_t nzero) {
  constexpr int NB = 1 << NBINS_LOG_SMALL;
  static_assert(NB == 1024, "one thread per bin");
  __shared__ uint32_t scan_tmp[1024 / 64 + 1];
  __shared__ uint32_t tot[NB];
  __shared__ unsigned int gmax[5];
  const int t = threadIdx.x;
  // every block clears its share of `zero`; block 0 also scans
  {
    const uint32_t nv = nzero / 4, per = (nv + gridDim.x - 1) / gridDim.x;
    const uint32_t z0 = blockIdx.x * per, z1 = min(nv, z0 + per);
    for (uint32_t i = z0 + t; i < z1; i += 1024)
      reinterpret_cast<uint4*>(zero)[i] = make_uint4(0u, 0u, 0u, 0u);
  }
  if (blockIdx.x != 0) return;
  if (t < 5) gmax[t] = 0u;
  uint32_t c[SMALL_SCAN_ROWS];
#pragma unroll
  for (int r = 0; r < SMALL_SCAN_ROWS; r++) c[r] = r < rows ? counts[(size_t)r * NB + t] : 0u;
  uint32_t run = 0;
#pragma unroll
  for (int r = 0; r < SMALL_SCAN_ROWS; r++) {
    if (r < rows) counts[(size_t)r * NB + t] = run;
    run += c[r];
  }
  tot[t] = run;
  uint32_t total;
  const uint32_t pre = block_exclusive_scan(run, scan_tmp, &total);  // barriers: tot, gmax set
  bin_base[t] = pre;
  if (t == 0) bin_base[NB] = total;
#pragma unroll
  for (int lg = 0; lg < 5; lg++) {
    const int g = 1 << lg;
    if ((t & (g - 1)) == 0) {
      uint32_t m = 0;
      for (int q = 0; q < g; q++) m += tot[t + q];
      atomicMax(&gmax[lg], m);
    }
  }
  __syncthreads();
  if (t == 0) {
    ctl->pe_total = total;
    ctl->ndefer = 0u;
    for (int lg = 0; lg < 5; lg++) ctl->maxg[lg] = gmax[lg];
  }
}

// Exclusive scan of the bin totals (one block of 1024 threads, of which the
// first scan_bins_threads<NBL>() hold the bins: thread t owns the BPT >= 16
// consecutive bins from t BPT, read and written as 16-byte vectors) and the
// largest total over aligned groups of 1, 2, 4, 8, 16 bins.  Also clears
// `zero` (nzero words) when given, with every thread: the level-0 |c|^2
// histogram of the merges that follow this count pass.
template <int NBL>
constexpr int scan_bins_threads() { return (1 << NBL) / 16 < 1024 ? (1 << NBL) / 16 : 1024; }
template <int NBL>
__global__ __launch_bounds__(1024) void k_scan_bins(const uint32_t* bin_total, uint32_t* bin_base,
                                                    Ctl* ctl, uint32_t* zero, uint32_t nzero,
                                                    unsigned long long spec_cap = 0ull,
                                                    unsigned int merge_cap = 0u) {
  constexpr int NB = 1 << NBL;
  constexpr int TH = scan_bins_threads<NBL>();
  constexpr int NWV = TH / 64;
  constexpr int BPT = NB / TH;
  static_assert(BPT >= 16 && BPT * TH == NB && BPT % 4 == 0 && NWV >= 1 && NWV <= 16,
                "k_scan_bins covers the bins with TH threads");
  __shared__ unsigned long long tmp[1024 / 64 + 1];
  __shared__ unsigned int gmax[16][5];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  // every thread of the block clears (nzero is a multiple of 4 and `zero`
  // 16-byte aligned: histogram replicas); the first TH threads, whole waves,
  // hold the bins, the others take part with empty bins
  for (uint32_t i = t; i < nzero / 4; i += blockDim.x)
    reinterpret_cast<uint4*>(zero)[i] = make_uint4(0u, 0u, 0u, 0u);
  const bool act = t < TH;
  uint32_t v[BPT];
  const uint4* src = reinterpret_cast<const uint4*>(bin_total) + (size_t)t * (BPT / 4);
#pragma unroll
  for (int q = 0; q < BPT / 4; q++) {
    const uint4 c = act ? src[q] : make_uint4(0u, 0u, 0u, 0u);
    v[4 * q] = c.x;
    v[4 * q + 1] = c.y;
    v[4 * q + 2] = c.z;
    v[4 * q + 3] = c.w;
  }
  unsigned long long s = 0;
#pragma unroll
  for (int k = 0; k < BPT; k++) s += v[k];
  unsigned int lm[5];
#pragma unroll
  for (int lg = 0; lg < 5; lg++) {
    const int g = 1 << lg;
    unsigned int best = 0;
#pragma unroll
    for (int k = 0; k < BPT; k += g) {
      unsigned long long acc = 0;
#pragma unroll
      for (int q = 0; q < g; q++) acc += v[k + q];
      const unsigned int a = acc > 0xFFFFFFFFull ? 0xFFFFFFFFu : (unsigned int)acc;
      best = a > best ? a : best;
    }
    // wave maximum, then one entry per wave
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const unsigned int o = __shfl_xor(best, d, 64);
      best = o > best ? o : best;
    }
    lm[lg] = best;
  }
  if (lane == 0)
#pragma unroll
    for (int lg = 0; lg < 5; lg++) gmax[wv][lg] = lm[lg];
  // block exclusive scan (u64)
  unsigned long long x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    unsigned long long y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wv] = x;
  __syncthreads();
  unsigned long long w = lane < NWV ? tmp[lane] : 0ull;
#pragma unroll
  for (int d = 1; d < 16; d <<= 1) {
    unsigned long long y = __shfl_up(w, d, 64);
    if (lane >= d) w += y;
  }
  const unsigned long long before = wv > 0 ? __shfl(w, wv - 1, 64) : 0ull;
  const unsigned long long total = __shfl(w, NWV - 1, 64);
  unsigned long long pre = before + x - s;
  uint4* dst = reinterpret_cast<uint4*>(bin_base) + (size_t)t * (BPT / 4);
#pragma unroll
  for (int q = 0; q < (act ? BPT / 4 : 0); q++) {
    uint4 o;
    o.x = (uint32_t)pre;
    pre += v[4 * q];
    o.y = (uint32_t)pre;
    pre += v[4 * q + 1];
    o.z = (uint32_t)pre;
    pre += v[4 * q + 2];
    o.w = (uint32_t)pre;
    pre += v[4 * q + 3];
    dst[q] = o;
  }
  if (t == 0) {
    bin_base[NB] = (uint32_t)total;
    ctl->pe_total = total;
    ctl->ndefer = 0u;
    if (total > 0xFFFFFFFFull) ctl->overflow |= 2u;
    for (int lg = 0; lg < 5; lg++) {
      unsigned int m = 0;
      for (int q = 0; q < NWV; q++) m = gmax[q][lg] > m ? gmax[q][lg] : m;
      ctl->maxg[lg] = m;
    }
    // a scatter already launched for a single pass laid out for spec_cap
    // records stands down unless the records fit and every bin fits a bucket
    if (spec_cap) ctl->spec_fail = (total > spec_cap || ctl->maxg[0] > merge_cap) ? 1u : 0u;
  }
}

// ---------------------------------------------------------------------------
// Linear combinations of canonical operators, merged without emission.  A
// term in canonical order (ascending mixed key, distinct strings) holds the
// strings of hash bucket b (the top F bits of the mixed key) as one
// contiguous run, so the merge can read each bucket straight from the terms:
// k_term_bounds finds the runs, k_check_sorted confirms the order of terms
// the engine did not write itself.
// ---------------------------------------------------------------------------
struct TermView {
  int n_terms;
  int F;  // 2^F buckets
  const uint64_t* tx[MAX_TERMS];
  const uint64_t* tz[MAX_TERMS];
  int64_t tcap[MAX_TERMS];
  int64_t tn[MAX_TERMS];
  const void* tc[MAX_TERMS];
  int tf32[MAX_TERMS];
  uint32_t tgroup[MAX_TERMS];
  const uint32_t* bounds;  // [n_terms][2^F + 1]: strings of term t in buckets below b
};

template <int W>
DEV Key<W> load_raw(const uint64_t* x, const uint64_t* z, int64_t cap, int64_t i) {
  Key<W> raw;
#pragma unroll
  for (int w = 0; w < W; w++) {
    raw.w[w] = x[(size_t)w * cap + i];
    raw.w[W + w] = z[(size_t)w * cap + i];
  }
  return raw;
}

// *flag |= 1 when the mixed keys of the n strings do not strictly ascend.
template <int W>
__global__ __launch_bounds__(256) void k_check_sorted(const uint64_t* x, const uint64_t* z,
                                                      int64_t cap, int64_t n, unsigned int* flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x + 1; i < n;
       i += (int64_t)gridDim.x * 256) {
    const Key<W> a = mix_key<W>(load_raw<W>(x, z, cap, i - 1));
    const Key<W> b = mix_key<W>(load_raw<W>(x, z, cap, i));
    bad = bad || key_cmp<W>(a, b) >= 0;
  }
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

// bounds[t][b], b = 0 .. 2^F: the first string of term t whose bucket is at
// least b (binary search over the canonical order; one thread per entry).
template <int W>
__global__ __launch_bounds__(256) void k_term_bounds(TermView v, uint32_t* bounds) {
  const int64_t nb1 = ((int64_t)1 << v.F) + 1;
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= nb1 * v.n_terms) return;
  const int t = (int)(id / nb1);
  const uint64_t b = (uint64_t)(id - (int64_t)t * nb1);
  int64_t lo = 0, hi = v.tn[t];
  if (v.F == 0) {
    lo = b ? hi : 0;
  } else {
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      const Key<W> m = mix_key<W>(load_raw<W>(v.tx[t], v.tz[t], v.tcap[t], mid));
      if ((m.w[0] >> (64 - v.F)) < b) lo = mid + 1;
      else hi = mid;
    }
  }
  bounds[id] = (uint32_t)lo;
}

struct MergeArgs {
  const uint32_t* bin_base;
  int nbins_log;  // hash bins of the call: 2^nbins_log per pass
  int g_log;
  int digit_shift;
  int pass_bits;
  uint32_t pass_id;
  int wide;
  const void* recs;
  const uint32_t* rsrc_wide;
  double2 alpha[MAX_GROUPS];
  int alpha_kind[MAX_GROUPS];
  int gkind[MAX_GROUPS];
  int mode;
  int single;  // one group, not Kahan: runs fold as plain sums
  int round32;
  int max_len;
  int use_eps;
  double eps2;
  const void* keep_mk;
  int n_keep;
  unsigned long long u_off;
  void* uk;
  double2* uc;
  uint32_t bucket_off;
  uint32_t* b_ubase;
  uint32_t* b_slots;
  uint32_t* b_surv;
  uint32_t* b_keep;
  uint32_t* b_unique;
  uint32_t* hist0;
  double2* norm_part;
  uint32_t* defer;  // buckets above the small variant's capacity (nullptr: none deferred)
  Ctl* ctl;
  TermView tv;      // direct merges: the canonical terms and their bucket runs
};

template <int W>
DEV bool keep_lookup(const Key<W>* keep, int n, const Key<W>& mk) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int c = key_cmp<W>(keep[mid], mk);
    if (c == 0) return true;
    if (c < 0) lo = mid + 1;
    else hi = mid;
  }
  return false;
}

DEV double2 apply_alpha(int kind, double2 alpha, double2 v) {
  if (kind == A_ONE) return v;
  if (kind == A_I) return make_double2(-v.y, v.x);
  if (kind == A_DIV) return make_double2(v.x / alpha.x, v.y / alpha.x);
  return cmul(alpha, v);
}

DEV double round_to_f32(double v) { return (double)(float)v; }

// The DIGIT_BITS + 32 bits of a mixed key that follow its first `shift`
// bits (0 <= shift < 64): the in-bucket digit on top, then 32 sort bits.
template <int W>
DEV uint64_t key_window(const Key<W>& m, int shift) {
  const uint64_t hi = shift ? ((m.w[0] << shift) | (m.w[1] >> (64 - shift))) : m.w[0];
  return hi >> (64 - DIGIT_BITS - 32);
}

// Rank of every record of the block inside its digit group by full
// (mixed key, source id) comparison, used when two distinct keys of a group
// share their 32 sort bits.  On entry mk/sx/sv hold the n records grouped by
// digit (ascending); on return they are in (key, source id) order.
template <int W, bool F32, int THREADS, int CAP>
DEV void merge_full_rank(Key<W>* mk, uint32_t* sx, RecV<F32>* sv, uint32_t n, int shift) {
  constexpr int PER = (CAP + THREADS - 1) / THREADS;
  Key<W> k[PER];
  uint32_t x[PER], pos[PER];
  typename std::conditional<F32, float, double>::type vx[PER], vy[PER];
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const uint32_t p = threadIdx.x + q * THREADS;
    pos[q] = p;
    if (p < n) {
      k[q] = mk[p];
      x[q] = sx[p];
      vx[q] = sv[p].x;
      vy[q] = sv[p].y;
      const uint32_t d = (uint32_t)(key_window<W>(k[q], shift) >> 32);
      // digit group [s0, s1): binary searches on the (ascending) digits
      uint32_t lo = 0, hi = p;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint32_t)(key_window<W>(mk[mid], shift) >> 32) < d) lo = mid + 1;
        else hi = mid;
      }
      const uint32_t s0 = lo;
      lo = p + 1;
      hi = n;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint32_t)(key_window<W>(mk[mid], shift) >> 32) <= d) lo = mid + 1;
        else hi = mid;
      }
      const uint32_t s1 = lo;
      uint32_t rank = 0;
      for (uint32_t r = s0; r < s1; r++) rank += key_src_less<W>(mk[r], sx[r], k[q], x[q]) ? 1u : 0u;
      pos[q] = s0 + rank;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const uint32_t p = threadIdx.x + q * THREADS;
    if (p < n) {
      mk[pos[q]] = k[q];
      sx[pos[q]] = x[q];
      sv[pos[q]].x = vx[q];
      sv[pos[q]].y = vy[q];
    }
  }
  __syncthreads();
}

// THREADS threads merge one bucket of at most CAP records.  MODE
// MERGE_GRID: block j merges bucket j; MERGE_SMALL: the same, but a bucket
// above CAP goes to the list a.defer instead (the small-bucket variant, 512
// threads, three blocks per CU by LDS); MERGE_LIST: the blocks merge the
// listed buckets.
enum MergeKind : int { MERGE_GRID = 0, MERGE_SMALL = 1, MERGE_LIST = 2 };
// DIRECT: the records of bucket j are the j-th runs of the canonical terms
// of a.tv (g_log = 0, no pass bits), read in place; source id = term group.
template <int W, bool F32, int THREADS, int CAP, int MODE, bool DIRECT = false>
__global__ __launch_bounds__(THREADS)
__attribute__((amdgpu_waves_per_eu(MODE == MERGE_SMALL ? 6 : 8))) void k_merge(MergeArgs a) {
  constexpr bool SMALL = MODE == MERGE_SMALL;
  using V = RecV<F32>;
  constexpr int PER = (CAP + THREADS - 1) / THREADS;
  constexpr int DPT = NDIGITS / THREADS;
  static_assert(SEL0_BINS == 2 * NDIGITS,
                "digit counts and the |c|^2 histogram (16-bit counters, two per word) share LDS");
  // Sort: a counting sort on the DIGIT_BITS key bits after the bucket bits,
  // then the rank of every record inside its digit group by a 64-bit sort
  // word (the next 32 key bits, then the source id), read from `swd` (which
  // aliases sv until the values are written).  mk / sx / sv then hold the
  // records in sorted order; dh holds the digit counts and starts, then the
  // level-0 histogram of |c|^2.  Two distinct keys of one digit group with
  // equal sort bits show up as adjacent entries with equal windows but
  // different keys; the block then ranks by full keys (merge_full_rank).
  __shared__ Key<W> mk[CAP];
  __shared__ __align__(16) V sv[CAP];
  static_assert(sizeof(V) >= sizeof(uint64_t), "sort words alias the values");
  uint64_t* const swd = reinterpret_cast<uint64_t*>(sv);
  __shared__ uint32_t sx[CAP];
  __shared__ int s_collide;
  __shared__ uint32_t s_pk;
  __shared__ uint32_t dh[NDIGITS];
  uint32_t* const h0 = dh;
  __shared__ uint32_t scan_tmp[THREADS / 64 + 1];
  __shared__ int s_gk[MAX_GROUPS], s_ak[MAX_GROUPS];
  __shared__ double2 s_al[MAX_GROUPS];
  __shared__ uint32_t sbb[17];
  constexpr int NHW = (CAP + 63) / 64;
  __shared__ uint64_t hmask[NHW];  // bit p: sorted position p starts a run of equal keys

  const int tid = threadIdx.x;
  auto bucket = [&](const uint32_t j) {
  const uint32_t gb = a.bucket_off + j;
  uint32_t b0, b1;
  // direct merges: start of the bucket's run in each term and the run's
  // first position in the bucket (tpre, ascending over the terms)
  uint32_t tst[DIRECT ? MAX_TERMS : 1], tpre[DIRECT ? MAX_TERMS : 1];
  if constexpr (DIRECT) {
    const uint32_t stride = (1u << a.tv.F) + 1u;
    b0 = 0u;
    b1 = 0u;
#pragma unroll
    for (int t = 0; t < MAX_TERMS; t++) {
      tst[t] = 0u;
      tpre[t] = 0xFFFFFFFFu;
      if (t < a.tv.n_terms) {
        const uint32_t s0 = a.tv.bounds[t * stride + j], s1 = a.tv.bounds[t * stride + j + 1];
        tst[t] = s0;
        tpre[t] = b1 - b0;
        b0 += s0;
        b1 += s1;
      }
    }
    if (a.ctl->unsorted) b1 = b0;  // the call is redone by emission
  } else {
    b0 = a.bin_base[j << a.g_log];
    b1 = a.bin_base[(j + 1) << a.g_log];
  }
  const uint32_t n = b1 - b0;
  const unsigned long long ub = a.u_off + b0;
  // direct merges: term, group and index of bucket position i (the last
  // term whose run starts at or before i; empty runs are passed over)
  struct TermPos {
    int t;
    int64_t e;
  };
  auto term_pos = [&](uint32_t i) -> TermPos {
    TermPos r{0, 0};
#pragma unroll
    for (int t = 0; t < (DIRECT ? MAX_TERMS : 1); t++)
      if (i >= tpre[t]) {
        r.t = t;
        r.e = (int64_t)tst[t] + (int64_t)(i - tpre[t]);
      }
    return r;
  };
  auto term_key = [&](const TermPos& q) -> Key<W> {
    return mix_key<W>(load_raw<W>(a.tv.tx[q.t], a.tv.tz[q.t], a.tv.tcap[q.t], q.e));
  };
  auto term_val = [&](const TermPos& q) -> V {
    V v;
    if (a.tv.tf32[q.t]) {
      const float2 f = reinterpret_cast<const float2*>(a.tv.tc[q.t])[q.e];
      v.x = f.x;
      v.y = f.y;
    } else {
      const double2 d = reinterpret_cast<const double2*>(a.tv.tc[q.t])[q.e];
      v.x = d.x;
      v.y = d.y;
    }
    return v;
  };
  if (n > (uint32_t)CAP) {
    if (SMALL) {  // left to the full-size variant
      if (tid == 0) a.defer[atomicAdd(&a.ctl->ndefer, 1u)] = j;
      return;
    }
    if (tid == 0) {
      atomicOr(&a.ctl->overflow, 1u);
      a.b_ubase[gb] = (uint32_t)ub;
      a.b_slots[gb] = 0;
      a.b_surv[gb] = 0;
      a.b_keep[gb] = 0;
      a.b_unique[gb] = 0;
    }
    return;
  }
  const Rec<W, F32>* recs = reinterpret_cast<const Rec<W, F32>*>(a.recs);
  const int F = a.nbins_log + a.pass_bits;
  const uint32_t ibits = (uint32_t)(F - 3);
  // Per record the digit, its rank among the digit's records, the source id
  // and the 32 sort bits stay in registers, and at W = 1 the order key; the
  // value (and a wider key) is read a second time, from cache, for the
  // sorted write, which keeps the kernel spill-free at 8 waves per SIMD.
  constexpr bool HOLD_KEY = W == 1;
  uint32_t dig[PER], rnk[PER], rsx[PER], swl[PER];
  uint64_t rkw[HOLD_KEY ? 2 * W : 1][PER];
  // one-word keys: the record loads are issued before the shared-memory
  // set-up, so that their latency overlaps it
  if constexpr (HOLD_KEY) {
#pragma unroll
    for (int k = 0; k < PER; k++) {
      const uint32_t i = tid + k * THREADS;
      rsx[k] = 0;
      if (i < n) {
        Key<W> m;
        if constexpr (DIRECT) {
          const TermPos q = term_pos(i);
          m = term_key(q);
          rsx[k] = a.tv.tgroup[q.t] << GROUP_SHIFT;
        } else {
          m = recs[b0 + i].k;
          if (a.wide) rsx[k] = a.rsrc_wide[b0 + i];
        }
#pragma unroll
        for (int q = 0; q < 2 * W; q++) rkw[q][k] = m.w[q];
      }
    }
  }
  for (int i = tid; i < NDIGITS; i += THREADS) dh[i] = 0u;
  if (tid < MAX_GROUPS) {
    s_gk[tid] = a.gkind[tid];
    s_ak[tid] = a.alpha_kind[tid];
    s_al[tid] = a.alpha[tid];
  }
  const int G = 1 << a.g_log;
  if (!DIRECT && tid <= G) sbb[tid] = a.bin_base[(j << a.g_log) + tid];
  if (tid == 0) {
    s_collide = 0;
    s_pk = 0u;
  }
  __syncthreads();

  // the record's order key: the bin bits that the source id displaced restored
  auto order_key = [&](uint32_t pos, const Key<W>& rk) -> Key<W> {
    int kb = 0;
    while (kb + 1 < G && sbb[kb + 1] <= pos) kb++;
    const uint64_t T = ((uint64_t)a.pass_id << a.nbins_log) | (uint64_t)((j << a.g_log) + kb);
    Key<W> m = rk;
    m.w[0] = (T << (64 - F)) | (rk.w[0] & (~0ull >> F));
    return m;
  };
  // sort word of record k: the 32 key bits after the digit, then the source id
  auto sort_word = [&](int k) -> uint64_t { return ((uint64_t)swl[k] << 32) | rsx[k]; };
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const uint32_t i = tid + k * THREADS;
    dig[k] = 0;
    rnk[k] = 0;
    swl[k] = 0;
    if (!HOLD_KEY) rsx[k] = 0;
    if (i < n) {
      const uint32_t pos = b0 + i;
      Key<W> m;
      if constexpr (HOLD_KEY) {
#pragma unroll
        for (int q = 0; q < 2 * W; q++) m.w[q] = rkw[q][k];
      } else if constexpr (DIRECT) {
        const TermPos q = term_pos(i);
        m = term_key(q);
        rsx[k] = a.tv.tgroup[q.t] << GROUP_SHIFT;
      } else {
        m = recs[pos].k;
        if (a.wide) rsx[k] = a.rsrc_wide[pos];
      }
      if constexpr (!DIRECT) {
        // the source id from the key's top bits, then the order key
        const uint32_t small = (uint32_t)(m.w[0] >> (64 - F));
        if (!a.wide) rsx[k] = ((small >> ibits) << GROUP_SHIFT) | (small & ((1u << ibits) - 1u));
        m = order_key(pos, m);
        if constexpr (HOLD_KEY) {
#pragma unroll
          for (int q = 0; q < 2 * W; q++) rkw[q][k] = m.w[q];
        }
      }
      const uint64_t win = key_window<W>(m, a.digit_shift);
      dig[k] = (uint32_t)(win >> 32);
      swl[k] = (uint32_t)win;
      rnk[k] = atomicAdd(&dh[dig[k]], 1u);
    }
  }
  __syncthreads();
  // digit starts (exclusive scan of the digit counts)
  {
    uint32_t loc[DPT], s = 0;
#pragma unroll
    for (int q = 0; q < DPT; q++) {
      loc[q] = dh[tid * DPT + q];
      s += loc[q];
    }
    uint32_t tot;
    uint32_t pre = block_exclusive_scan(s, scan_tmp, &tot);
#pragma unroll
    for (int q = 0; q < DPT; q++) {
      dh[tid * DPT + q] = pre;
      pre += loc[q];
    }
  }
  __syncthreads();
  // sort words in digit-group order
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const uint32_t i = tid + k * THREADS;
    if (i < n) swd[dh[dig[k]] + rnk[k]] = sort_word(k);
  }
  __syncthreads();
  // Final position of every record: its digit group's start plus the number of
  // group members with a smaller sort word (equal words: earlier entry first).
  uint32_t fpos[PER];
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const uint32_t i = tid + k * THREADS;
    fpos[k] = 0;
    if (i < n) {
      const uint32_t s0 = dh[dig[k]];
      const uint32_t s1 = dig[k] + 1 < (uint32_t)NDIGITS ? dh[dig[k] + 1] : n;
      const uint32_t me = s0 + rnk[k];
      const uint64_t w = sort_word(k);
      uint32_t rank = 0;
      uint32_t p = s0;
      for (; p + 4 <= s1; p += 4) {
        const uint64_t w0 = swd[p], w1 = swd[p + 1], w2 = swd[p + 2], w3 = swd[p + 3];
        rank += ((w0 < w) | ((w0 == w) & (p < me))) ? 1u : 0u;
        rank += ((w1 < w) | ((w1 == w) & (p + 1 < me))) ? 1u : 0u;
        rank += ((w2 < w) | ((w2 == w) & (p + 2 < me))) ? 1u : 0u;
        rank += ((w3 < w) | ((w3 == w) & (p + 3 < me))) ? 1u : 0u;
      }
      for (; p < s1; p++) {
        const uint64_t w0 = swd[p];
        rank += ((w0 < w) | ((w0 == w) & (p < me))) ? 1u : 0u;
      }
      fpos[k] = s0 + rank;
    }
  }
  __syncthreads();
  // keys, sources and values in sorted order; the digit counts become the
  // level-0 |c|^2 histogram (16-bit counters, two per word)
  if (a.mode == M_PLAIN)
    for (int i = tid; i < NDIGITS; i += THREADS) h0[i] = 0u;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const uint32_t i = tid + k * THREADS;
    if (i < n) {
      if constexpr (HOLD_KEY) {
        Key<W> m;
#pragma unroll
        for (int q = 0; q < 2 * W; q++) m.w[q] = rkw[q][k];
        mk[fpos[k]] = m;
        if constexpr (DIRECT) sv[fpos[k]] = term_val(term_pos(i));
        else sv[fpos[k]] = recs[b0 + i].v;  // second read (cache)
      } else if constexpr (DIRECT) {
        const TermPos q = term_pos(i);  // second read (cache)
        mk[fpos[k]] = term_key(q);
        sv[fpos[k]] = term_val(q);
      } else {
        const Rec<W, F32> r = recs[b0 + i];  // second read (cache)
        mk[fpos[k]] = order_key(b0 + i, r.k);
        sv[fpos[k]] = r.v;
      }
      sx[fpos[k]] = rsx[k];
    }
  }
  __syncthreads();

  const Key<W>* keep = reinterpret_cast<const Key<W>*>(a.keep_mk);
  // Fold the run [p, q) of equal keys: groups in ascending id, a SUM group
  // adds its contributions in ascending source index, then
  // acc = g0, acc = fl(acc + g1), ... after scaling each group by its alpha.
  auto fold = [&](uint32_t p, uint32_t q, double2& out) -> bool {
    if (a.single) {
      // one group: the sequential sum of the run, then the group's alpha
      const int g = (int)(sx[p] >> GROUP_SHIFT);
      const V v0 = sv[p];
      double sr = (double)v0.x, si = (double)v0.y;
      uint32_t r = p + 1;
      for (; r + 4 <= q; r += 4) {
        const V v1 = sv[r], v2 = sv[r + 1], v3 = sv[r + 2], v4 = sv[r + 3];
        sr = sr + (double)v1.x;
        si = si + (double)v1.y;
        sr = sr + (double)v2.x;
        si = si + (double)v2.y;
        sr = sr + (double)v3.x;
        si = si + (double)v3.y;
        sr = sr + (double)v4.x;
        si = si + (double)v4.y;
      }
      for (; r < q; r++) {
        const V v1 = sv[r];
        sr = sr + (double)v1.x;
        si = si + (double)v1.y;
      }
      double2 acc = apply_alpha(s_ak[g], s_al[g], make_double2(sr, si));
      if (a.round32) acc = make_double2(round_to_f32(acc.x), round_to_f32(acc.y));
      out = acc;
      return !is_zero(acc);
    }
    bool present = false;
    double2 acc = make_double2(0.0, 0.0);
    int cur = -1;
    double2 gs = make_double2(0.0, 0.0);
    float kr = 0.f, kcr = 0.f, ki = 0.f, kci = 0.f;  // Kahan state (FP32 records only)
    auto finish = [&]() {
      double2 gv = gs;
      if constexpr (F32) {
        if (s_gk[cur] == G_SUM_KAHAN32)
          gv = make_double2((double)kr - (double)kcr, (double)ki - (double)kci);
      }
      gv = apply_alpha(s_ak[cur], s_al[cur], gv);
      if (!present) acc = gv;
      else acc = make_double2(acc.x + gv.x, acc.y + gv.y);
      present = true;
    };
    constexpr int FU = 2;  // run entries loaded per step (LDS loads issued together)
    for (uint32_t r0 = p; r0 < q; r0 += FU) {
     uint32_t gx[FU];
     V vv[FU];
#pragma unroll
     for (int u = 0; u < FU; u++)
       if (r0 + u < q) {
         gx[u] = sx[r0 + u];
         vv[u] = sv[r0 + u];
       }
#pragma unroll
     for (int u = 0; u < FU; u++) {
      if (r0 + u >= q) break;
      const int g = (int)(gx[u] >> GROUP_SHIFT);
      const V v = vv[u];
      const bool kahan = F32 && s_gk[g] == G_SUM_KAHAN32;
      if (g != cur) {
        if (cur >= 0) finish();
        cur = g;
        if (kahan) {
          kr = 0.f; kcr = 0.f; ki = 0.f; kci = 0.f;
          kahan_add(kr, kcr, (float)v.x);
          kahan_add(ki, kci, (float)v.y);
        } else {
          gs = make_double2((double)v.x, (double)v.y);
        }
      } else {
        if (kahan) {
          kahan_add(kr, kcr, (float)v.x);
          kahan_add(ki, kci, (float)v.y);
        } else {
          gs = make_double2(gs.x + (double)v.x, gs.y + (double)v.y);
        }
      }
     }
    }
    if (cur >= 0) finish();
    if (a.round32) acc = make_double2(round_to_f32(acc.x), round_to_f32(acc.y));
    out = acc;
    return !is_zero(acc);
  };

  // Head bits of the sorted positions (a position starts a run of equal keys).
  Key<W>* uk = reinterpret_cast<Key<W>*>(a.uk) + ub;
  double2* uc = a.uc + ub;
  uint32_t kc = 0, nzu = 0;
  const uint32_t nround = (n + THREADS - 1) / THREADS;
  const uint32_t nwords = (n + 63) / 64;
  // the window (digit and sort bits) as masks of the first two key words:
  // two keys share it when their XOR has none of the masked bits
  constexpr int WB = DIGIT_BITS + 32;
  const int wsh = a.digit_shift;
  const uint64_t wm0 = wsh + WB <= 64 ? (((1ull << WB) - 1ull) << (64 - wsh - WB)) : (~0ull >> wsh);
  const uint64_t wm1 = wsh + WB <= 64 ? 0ull : ~(~0ull >> (wsh + WB - 64));
  for (uint32_t r = 0; r < nround; r++) {
    const uint32_t p = r * THREADS + tid;
    bool head = false;
    if (p < n) {
      head = p == 0;
      if (p > 0) {
        const Key<W> k0 = mk[p - 1], k1 = mk[p];
        head = !key_eq<W>(k0, k1);
        if (head && ((k0.w[0] ^ k1.w[0]) & wm0) == 0 && ((k0.w[1] ^ k1.w[1]) & wm1) == 0)
          s_collide = 1;
      }
    }
    const uint64_t m = __ballot(head);
    if ((tid & 63) == 0 && (p >> 6) < (uint32_t)NHW) hmask[p >> 6] = m;
  }
  __syncthreads();
  if (s_collide) {
    // rare: distinct keys with equal sort bits; rank again by full keys
    merge_full_rank<W, F32, THREADS, CAP>(mk, sx, sv, n, a.digit_shift);
    for (uint32_t r = 0; r < nround; r++) {
      const uint32_t p = r * THREADS + tid;
      const bool head = p < n && (p == 0 || !key_eq<W>(mk[p - 1], mk[p]));
      const uint64_t m = __ballot(head);
      if ((tid & 63) == 0 && (p >> 6) < (uint32_t)NHW) hmask[p >> 6] = m;
    }
    __syncthreads();
  }
  // Thread t owns the `per` consecutive sorted positions [per t, per t + per)
  // (per = ceil(n / threads) <= PER, so the work spreads over all waves): it
  // folds the runs that start there (a run may reach into the next threads'
  // positions), applies the filters (plain mode), and one block scan places
  // every survivor in sorted order.
  static_assert(PER * THREADS >= CAP, "every position has an owner");
  const uint32_t per = (n + THREADS - 1) / THREADS;
  double2 fv[PER];
  uint32_t smask = 0;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const uint32_t p = tid * per + k;
    fv[k] = make_double2(0.0, 0.0);
    if ((uint32_t)k < per && p < n && ((hmask[p >> 6] >> (p & 63)) & 1ull)) {
      // end of the run: the next head bit after p (or n)
      uint32_t q = n;
      const uint32_t w = p >> 6, bp = p & 63;
      const uint64_t rest = bp == 63 ? 0ull : (hmask[w] >> (bp + 1));
      if (rest) {
        q = p + 1 + (uint32_t)__builtin_ctzll(rest);
      } else {
        for (uint32_t ww = w + 1; ww < nwords; ww++)
          if (hmask[ww]) {
            q = ww * 64 + (uint32_t)__builtin_ctzll(hmask[ww]);
            break;
          }
      }
      if (q > n) q = n;
      double2 v;
      // direct merges apply the length cap here (emission applies it to
      // records before they reach a bucket)
      const bool too_long = DIRECT && a.mode == M_PLAIN && a.max_len > 0 &&
                            key_length<W>(unmix_key<W>(mk[p])) > a.max_len;
      if (!too_long && fold(p, q, v)) {
        nzu++;
        bool surv = true;
        if (a.mode != M_LANCZOS) {
          // the length cap was applied when the records were emitted
          if (a.use_eps && !(weight2(v) >= a.eps2)) surv = false;
          if (surv) {
            const bool isk = a.n_keep ? keep_lookup<W>(keep, a.n_keep, mk[p]) : false;
            if (isk) kc++;
            else {
              // 16-bit counters (a bucket holds < 2^16 records), two per word
              const uint32_t hb = (uint32_t)((uint64_t)__double_as_longlong(weight2(v)) >> SEL0_SHIFT);
              atomicAdd(&h0[hb >> 1], 1u << ((hb & 1u) << 4));
            }
          }
        }
        if (surv) {
          fv[k] = v;
          smask |= 1u << k;
        }
      }
    }
  }
  // block totals of the keep count and the nonzero count (both <= CAP: one
  // packed word), added per wave before the scan's barriers
  {
    uint32_t pk = (kc << 16) | nzu;
    for (int d = 32; d >= 1; d >>= 1) pk += __shfl_down(pk, d, 64);
    if ((tid & 63) == 0) atomicAdd(&s_pk, pk);
  }
  uint32_t tot_cnt;
  {
    uint32_t o = block_exclusive_scan((uint32_t)__popc(smask), scan_tmp, &tot_cnt);
    // U keeps order keys; raw strings are restored where needed
#pragma unroll
    for (int k = 0; k < PER; k++)
      if ((smask >> k) & 1u) {
        uk[o] = mk[tid * per + k];
        uc[o] = fv[k];
        o++;
      }
  }
  // the scan's barriers have ordered every histogram and s_pk update
  const uint32_t tot_kc = s_pk >> 16, tot_nzu = s_pk & 0xFFFFu;
  if (a.mode == M_PLAIN) {
    // word i of the LDS histogram holds bins 2i (low half) and 2i + 1
    uint32_t* hrep = a.hist0 + (size_t)(j % HREP) * SEL0_BINS;
    for (int i = tid; i < NDIGITS; i += THREADS) {
      const uint32_t w = h0[i];
      if (w & 0xFFFFu) atomicAdd(&hrep[2 * i], w & 0xFFFFu);
      if (w >> 16) atomicAdd(&hrep[2 * i + 1], w >> 16);
    }
  }
  if (tid == 0) {
    a.b_ubase[gb] = (uint32_t)ub;
    a.b_slots[gb] = tot_cnt;
    a.b_surv[gb] = tot_cnt;
    a.b_keep[gb] = tot_kc;
    a.b_unique[gb] = tot_nzu;
  }
  };
  if constexpr (MODE != MERGE_LIST) {
    bucket(blockIdx.x);
  } else {
    const uint32_t nd = *reinterpret_cast<volatile unsigned int*>(&a.ctl->ndefer);
    for (uint32_t it = blockIdx.x; it < nd; it += gridDim.x) {
      bucket(a.defer[it]);
      __syncthreads();  // the next bucket reuses the shared arrays
    }
  }
}

// Coefficient of the identity string (all mask words zero) of an operator
// with distinct strings: Tr(A)/2^N.  `res` (two doubles) starts at zero; at
// most one thread writes it.
__global__ __launch_bounds__(256) void k_trace(const uint64_t* x, const uint64_t* z, int64_t cap,
                                               int64_t n, int W, const void* coef, int f32,
                                               double* res) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    uint64_t s = 0;
    for (int w = 0; w < W; w++) s |= x[(size_t)w * cap + i] | z[(size_t)w * cap + i];
    if (s == 0) {
      if (f32) {
        const float2 v = reinterpret_cast<const float2*>(coef)[i];
        res[0] = (double)v.x;
        res[1] = (double)v.y;
      } else {
        const double2 v = reinterpret_cast<const double2*>(coef)[i];
        res[0] = v.x;
        res[1] = v.y;
      }
    }
  }
}

// Lanczos: double-double partial of sum |c|^2 over one bucket of the merged,
// untruncated O'_n (fixed reduction order).
__global__ __launch_bounds__(256) void k_norm_bucket(const uint32_t* b_ubase,
                                                     const uint32_t* b_slots, const double2* uc,
                                                     double2* part) {
  __shared__ double rh[4], rl[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint32_t b = blockIdx.x;
  const uint32_t ub = b_ubase[b], ns = b_slots[b];
  dd s = dd_zero();
  for (uint32_t i = tid; i < ns; i += 256) s = dd_add(s, weight2(uc[ub + i]));
  for (int d = 32; d >= 1; d >>= 1) {
    dd o;
    o.hi = __shfl_down(s.hi, d, 64);
    o.lo = __shfl_down(s.lo, d, 64);
    if (lane < d) s = dd_add(s, o);
  }
  if (lane == 0) {
    rh[wv] = s.hi;
    rl[wv] = s.lo;
  }
  __syncthreads();
  if (tid == 0) {
    dd t = {rh[0], rl[0]};
    for (int w = 1; w < 4; w++) t = dd_add(t, dd{rh[w], rl[w]});
    part[b] = make_double2(t.hi, t.lo);
  }
}

// k_norm_bucket for translation-symmetric operators: each merged unique
// weighted by its stabilizer count (the norm of sum_k T_k(A) over N).
template <int W>
__global__ __launch_bounds__(256) void k_norm_bucket_ts(const uint32_t* b_ubase,
                                                        const uint32_t* b_slots, const void* uk_,
                                                        const double2* uc, int N, double2* part) {
  __shared__ double rh[4], rl[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint32_t b = blockIdx.x;
  const uint32_t ub = b_ubase[b], ns = b_slots[b];
  const Key<W>* uk = reinterpret_cast<const Key<W>*>(uk_) + ub;
  dd s = dd_zero();
  for (uint32_t i = tid; i < ns; i += 256) {
    const Key<W> raw = unmix_key<W>(uk[i]);
    const int st = ts_stabilizers<W>(raw.w, raw.w + W, N);
    const double w2 = weight2(uc[ub + i]);
    for (int r = 0; r < st; r++) s = dd_add(s, w2);
  }
  for (int d = 32; d >= 1; d >>= 1) {
    dd o;
    o.hi = __shfl_down(s.hi, d, 64);
    o.lo = __shfl_down(s.lo, d, 64);
    if (lane < d) s = dd_add(s, o);
  }
  if (lane == 0) {
    rh[wv] = s.hi;
    rl[wv] = s.lo;
  }
  __syncthreads();
  if (tid == 0) {
    dd t = {rh[0], rl[0]};
    for (int w = 1; w < 4; w++) t = dd_add(t, dd{rh[w], rl[w]});
    part[b] = make_double2(t.hi, t.lo);
  }
}

// Totals of the per-bucket counters (one block): slots, survivors, keep-set
// survivors, nonzero uniques.
__global__ __launch_bounds__(1024) void k_bucket_totals(const uint32_t* b_slots,
                                                        const uint32_t* b_surv,
                                                        const uint32_t* b_keep,
                                                        const uint32_t* b_unique, uint32_t nb,
                                                        Ctl* ctl) {
  __shared__ unsigned long long red[4][16];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  unsigned long long v[4] = {0, 0, 0, 0};
  for (uint32_t b = t; b < nb; b += 1024) {
    v[0] += b_slots[b];
    v[1] += b_surv[b];
    v[2] += b_keep[b];
    if (b_unique) v[3] += b_unique[b];
  }
  for (int q = 0; q < 4; q++) {
    unsigned long long x = v[q];
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_down(x, d, 64);
    if (lane == 0) red[q][wv] = x;
  }
  __syncthreads();
  if (t == 0) {
    unsigned long long tot[4] = {0, 0, 0, 0};
    for (int q = 0; q < 4; q++)
      for (int w = 0; w < 16; w++) tot[q] += red[q][w];
    ctl->u_slots = tot[0];
    ctl->surv_total = tot[1];
    ctl->keep_total = tot[2];
    if (b_unique) ctl->u_unique = tot[3];
  }
}

// Deterministic double-double sum of n partials (one block).
__global__ __launch_bounds__(1024) void k_reduce_dd(const double2* part, uint32_t n, double* out) {
  // four independent double-double chains per thread (partials i, i + 1024,
  // i + 2048, i + 3072 of every 4096), combined in a fixed order
  __shared__ double rh[16], rl[16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  dd s[4] = {dd_zero(), dd_zero(), dd_zero(), dd_zero()};
  for (uint32_t i0 = 0; i0 < n; i0 += 4096) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const uint32_t i = i0 + q * 1024 + tid;
      if (i < n) s[q] = dd_add(s[q], dd{part[i].x, part[i].y});
    }
  }
  dd t = dd_add(dd_add(s[0], s[1]), dd_add(s[2], s[3]));
  for (int d = 32; d >= 1; d >>= 1) {
    dd o;
    o.hi = __shfl_down(t.hi, d, 64);
    o.lo = __shfl_down(t.lo, d, 64);
    if (lane < d) t = dd_add(t, o);
  }
  if (lane == 0) {
    rh[wv] = t.hi;
    rl[wv] = t.lo;
  }
  __syncthreads();
  if (tid == 0) {
    dd u = {rh[0], rl[0]};
    for (int w = 1; w < 16; w++) u = dd_add(u, dd{rh[w], rl[w]});
    out[0] = u.hi;
    out[1] = u.lo;
  }
}

// Lanczos: divide the merged O'_n by b_n (IEEE division), then apply the
// plain-mode filters on the FP64 quotient (FP32 outputs are rounded when
// written); dropped strings become exact zeros in place.
struct ScaleArgs {
  const uint32_t* b_ubase;
  const uint32_t* b_slots;
  uint32_t* b_surv;
  uint32_t* b_keep;
  void* uk;
  double2* uc;
  const double* norm2;  // ||O'_n||^2, written by the norm reduction
  double floor_b;       // b_n at or below this is a breakdown: nothing survives
  int round32;
  int max_len;
  int use_eps;
  double eps2;
  const void* keep_mk;
  int n_keep;
  uint32_t* hist0;
  Ctl* ctl;
};

template <int W>
__global__ __launch_bounds__(256) void k_scale_filter(ScaleArgs a) {
  __shared__ uint32_t h0[SEL0_BINS];
  __shared__ uint32_t rs[4], rk[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint32_t b = blockIdx.x;
  for (int i = tid; i < SEL0_BINS; i += 256) h0[i] = 0u;
  __syncthreads();
  const uint32_t ub = a.b_ubase[b], ns = a.b_slots[b];
  const Key<W>* uk = reinterpret_cast<const Key<W>*>(a.uk) + ub;
  double2* uc = a.uc + ub;
  const Key<W>* keep = reinterpret_cast<const Key<W>*>(a.keep_mk);
  // b_n = sqrt(||O'_n||^2), correctly rounded as on the host, which reads the
  // same norm with the output size and reports the breakdown
  const double bn = sqrt(*a.norm2);
  const bool brk = !(bn > a.floor_b);
  uint32_t surv = 0, kc = 0;
  for (uint32_t i = tid; i < ns; i += 256) {
    double2 v = uc[i];
    v = make_double2(v.x / bn, v.y / bn);
    // FP32 storage: a string whose stored value would be an exact zero is
    // dropped; every other decision (cutoff, top-M) is taken on the FP64
    // quotient, which the output write rounds to FP32
    bool ok = !brk && (a.round32 ? !is_zero(make_double2(round_to_f32(v.x), round_to_f32(v.y)))
                                 : !is_zero(v));
    const Key<W> mk = uk[i];
    if (ok && a.max_len > 0 && key_length<W>(unmix_key<W>(mk)) > a.max_len) ok = false;
    if (ok && a.use_eps && !(weight2(v) >= a.eps2)) ok = false;
    if (ok) {
      surv++;
      bool isk = a.n_keep ? keep_lookup<W>(keep, a.n_keep, mk) : false;
      if (isk) kc++;
      else atomicAdd(&h0[(uint32_t)((uint64_t)__double_as_longlong(weight2(v)) >> SEL0_SHIFT)], 1u);
    } else {
      v = make_double2(0.0, 0.0);
    }
    uc[i] = v;
  }
  for (int d = 32; d >= 1; d >>= 1) {
    surv += __shfl_down(surv, d, 64);
    kc += __shfl_down(kc, d, 64);
  }
  if (lane == 0) {
    rs[wv] = surv;
    rk[wv] = kc;
  }
  __syncthreads();
  uint32_t* hrep = a.hist0 + (size_t)(b % HREP) * SEL0_BINS;
  for (int i = tid; i < SEL0_BINS; i += 256)
    if (h0[i]) atomicAdd(&hrep[i], h0[i]);
  if (tid == 0) {
    a.b_surv[b] = rs[0] + rs[1] + rs[2] + rs[3];
    a.b_keep[b] = rk[0] + rk[1] + rk[2] + rk[3];
  }
}

// ---------------------------------------------------------------------------
// Top-M selection: exact radix select over the composite ordering key
// (|c|^2 bits, then the complemented key words x[W-1]..x[0], z[W-1]..z[0]):
// larger composite = kept first.  Digit 0 = the top 13 bits of |c|^2 (sign,
// always 0, the 11 exponent bits and the first mantissa bit: 4096 bins),
// digit L >= 1 = the 12 bits at position 12L + 1 of the composite bit string.
// ---------------------------------------------------------------------------
template <int W>
DEV void composite(double2 v, const Key<W>& raw, uint64_t* c) {
  c[0] = (uint64_t)__double_as_longlong(weight2(v));
#pragma unroll
  for (int i = 0; i < W; i++) {
    c[1 + i] = ~raw.w[W - 1 - i];
    c[1 + W + i] = ~raw.w[2 * W - 1 - i];
  }
}

template <int W>
DEV uint32_t comp_digit(const uint64_t* c, int level) {
  if (level == 0) return (uint32_t)(c[0] >> SEL0_SHIFT);
  const int p = 12 * level + (64 - SEL0_SHIFT - 12);  // 12-bit digits after the level-0 bits
  const int wi = p >> 6, off = p & 63;
  constexpr int NW = 1 + 2 * W;
  const uint64_t hi = wi < NW ? c[wi] : 0ull;
  const uint64_t lo = wi + 1 < NW ? c[wi + 1] : 0ull;
  const uint64_t v = off ? ((hi << off) | (lo >> (64 - off))) : hi;
  return (uint32_t)(v >> 52);
}

template <int W>
DEV int comp_cmp(const uint64_t* a, const uint64_t* b) {
#pragma unroll
  for (int i = 0; i < 1 + 2 * W; i++)
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return 0;
}

// Sum of the HREP replicas of a select histogram.
__global__ void k_hist_reduce(const uint32_t* rep, int nbins, uint32_t* sum) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  uint32_t s = 0;
#pragma unroll 8
  for (int r = 0; r < HREP; r++) s += rep[(size_t)r * nbins + b];
  sum[b] = s;
}

// Pick the bin holding the K-th largest: K from ctl->sel_K (1-based).
__global__ __launch_bounds__(1024) void k_select(const uint32_t* hist, int nbins, Ctl* ctl) {
  __shared__ unsigned long long tmp[17];
  __shared__ unsigned long long Ks;
  const int t = threadIdx.x;
  if (t == 0) Ks = ctl->sel_K;
  const int per = nbins / 1024;  // nbins is 2048 or 4096
  // thread t owns bins [nbins - (t+1)*per, nbins - t*per), scanned high to low
  const int hiB = nbins - t * per;
  unsigned int hv[4] = {0u, 0u, 0u, 0u};
  for (int q = 1; q <= per; q++) hv[q - 1] = hist[hiB - q];
  unsigned long long s = 0;
  for (int q = 1; q <= per; q++) s += hv[q - 1];
  const int lane = t & 63, wv = t >> 6;
  unsigned long long x = s;
  for (int d = 1; d < 64; d <<= 1) {
    unsigned long long y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wv] = x;
  __syncthreads();
  if (t == 0) {
    unsigned long long run = 0;
    for (int i = 0; i < 16; i++) {
      unsigned long long q = tmp[i];
      tmp[i] = run;
      run += q;
    }
  }
  __syncthreads();
  const unsigned long long K = Ks;
  unsigned long long cum = tmp[wv] + x - s;  // records in bins above this thread's
  for (int q = 1; q <= per; q++) {
    const int b = hiB - q;
    const unsigned long long h = hv[q - 1];
    if (cum < K && K <= cum + h) {
      ctl->sel_digit = (unsigned int)b;
      ctl->sel_K = K - cum;
      ctl->sel_count = h;
    }
    cum += h;
  }
}

struct SelArgs {
  const uint32_t* b_ubase;
  const uint32_t* b_slots;
  uint32_t* b_abv;
  uint32_t* b_bcnt;
  const void* uk;
  const double2* uc;
  const void* keep_mk;
  int n_keep;
  uint32_t nbk;
  // candidate lists: the entries of bucket b sit at [b_ubase[b], b_ubase[b] + cc[b])
  const uint32_t* list_in;
  const uint32_t* cc_in;
  uint32_t* list_out;
  uint32_t* cc_out;
  int level;
  uint32_t* hist;  // histogram of the next digit (nullable)
  Ctl* ctl;
};

// Level 1: one block per bucket, full pass over its U slots.  Counts the
// non-keep survivors whose digit 0 is above the chosen bin, collects the
// chosen bin's records (in bucket order) and histograms their digit 1.
template <int W>
__global__ __launch_bounds__(256) void k_level1(SelArgs a) {
  __shared__ uint32_t h[SEL_BINS];
  __shared__ uint32_t ra[4];
  __shared__ uint32_t scan_tmp[256 / 64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint32_t b = blockIdx.x;
  for (int i = tid; i < SEL_BINS; i += 256) h[i] = 0u;
  __syncthreads();
  const uint32_t D = a.ctl->sel_digit;
  const uint32_t ub = a.b_ubase[b], ns = a.b_slots[b];
  const Key<W>* uk = reinterpret_cast<const Key<W>*>(a.uk) + ub;
  const double2* uc = a.uc + ub;
  const Key<W>* keep = reinterpret_cast<const Key<W>*>(a.keep_mk);
  uint32_t abv = 0, nout = 0;
  const uint32_t nround = (ns + 255) / 256;
  for (uint32_t r = 0; r < nround; r++) {
    const uint32_t i = r * 256 + tid;
    bool cand = false;
    uint64_t c[1 + 2 * W];
    if (i < ns) {
      const double2 v = uc[i];
      if (!is_zero(v)) {
        const Key<W> mk = uk[i];
        const bool isk = a.n_keep ? keep_lookup<W>(keep, a.n_keep, mk) : false;
        if (!isk) {
          composite<W>(v, unmix_key<W>(mk), c);
          const uint32_t d0 = comp_digit<W>(c, 0);
          if (d0 > D) abv++;
          else if (d0 == D) cand = true;
        }
      }
    }
    uint32_t tot;
    const uint32_t pos = block_exclusive_scan(cand ? 1u : 0u, scan_tmp, &tot);
    if (cand) {
      a.list_out[ub + nout + pos] = ub + i;
      atomicAdd(&h[comp_digit<W>(c, 1)], 1u);
    }
    nout += tot;
  }
  for (int d = 32; d >= 1; d >>= 1) abv += __shfl_down(abv, d, 64);
  if (lane == 0) ra[wv] = abv;
  __syncthreads();
  uint32_t* hrep = a.hist + (size_t)(b % HREP) * SEL_BINS;
  for (int i = tid; i < SEL_BINS; i += 256)
    if (h[i]) atomicAdd(&hrep[i], h[i]);
  if (tid == 0) {
    a.b_abv[b] = ra[0] + ra[1] + ra[2] + ra[3];
    a.cc_out[b] = nout;
  }
}

// Level L >= 1, one block per bucket over its candidates: keep those whose
// digit L equals the chosen bin, histogram their digit L+1 (if hist given).
template <int W>
__global__ __launch_bounds__(256) void k_cand_level(SelArgs a) {
  __shared__ uint32_t h[SEL_BINS];
  __shared__ uint32_t scan_tmp[256 / 64 + 1];
  const int tid = threadIdx.x;
  const uint32_t b = blockIdx.x;
  const uint32_t n = a.cc_in[b];
  if (n == 0) {
    if (tid == 0) a.cc_out[b] = 0;
    return;
  }
  const bool with_hist = a.hist != nullptr;
  if (with_hist)
    for (int i = tid; i < SEL_BINS; i += 256) h[i] = 0u;
  __syncthreads();
  const uint32_t D = a.ctl->sel_digit;
  const uint32_t ub = a.b_ubase[b];
  const Key<W>* ukb = reinterpret_cast<const Key<W>*>(a.uk);
  uint32_t nout = 0;
  const uint32_t nround = (n + 255) / 256;
  for (uint32_t r = 0; r < nround; r++) {
    const uint32_t i = r * 256 + tid;
    bool keepit = false;
    uint64_t c[1 + 2 * W];
    uint32_t ui = 0;
    if (i < n) {
      ui = a.list_in[ub + i];
      composite<W>(a.uc[ui], unmix_key<W>(ukb[ui]), c);
      keepit = comp_digit<W>(c, a.level) == D;
    }
    uint32_t tot;
    const uint32_t pos = block_exclusive_scan(keepit ? 1u : 0u, scan_tmp, &tot);
    if (keepit) {
      a.list_out[ub + nout + pos] = ui;
      if (with_hist) atomicAdd(&h[comp_digit<W>(c, a.level + 1)], 1u);
    }
    nout += tot;
  }
  __syncthreads();
  if (with_hist) {
    uint32_t* hrep = a.hist + (size_t)(b % HREP) * SEL_BINS;
    for (int i = tid; i < SEL_BINS; i += 256)
      if (h[i]) atomicAdd(&hrep[i], h[i]);
  }
  if (tid == 0) a.cc_out[b] = nout;
}

// Final level (one block): every entry of list_in belongs to the chosen bin
// and there are at most FINISH_CAP of them; the entry of rank K-1
// (descending composite) is the threshold T.
template <int W>
__global__ __launch_bounds__(1024) void k_finish(SelArgs a) {
  constexpr int NW = 1 + 2 * W;
  __shared__ uint64_t cs[FINISH_CAP][NW];
  __shared__ unsigned int m;
  const int tid = threadIdx.x;
  if (tid == 0) m = 0;
  __syncthreads();
  const Key<W>* ukb = reinterpret_cast<const Key<W>*>(a.uk);
  for (uint32_t b = tid; b < a.nbk; b += 1024) {
    const uint32_t n = a.cc_in[b];
    if (!n) continue;
    const uint32_t ub = a.b_ubase[b];
    for (uint32_t k = 0; k < n; k++) {
      const uint32_t ui = a.list_in[ub + k];
      uint64_t c[NW];
      composite<W>(a.uc[ui], unmix_key<W>(ukb[ui]), c);
      const unsigned int p = atomicAdd(&m, 1u);
      if (p < FINISH_CAP)
        for (int q = 0; q < NW; q++) cs[p][q] = c[q];
    }
  }
  __syncthreads();
  const unsigned int mm = m < FINISH_CAP ? m : FINISH_CAP;
  const unsigned long long K = a.ctl->sel_K;
  for (unsigned int i = tid; i < mm; i += 1024) {
    unsigned int rank = 0;
    for (unsigned int k = 0; k < mm; k++) rank += comp_cmp<W>(cs[k], cs[i]) > 0 ? 1u : 0u;
    if ((unsigned long long)rank + 1 == K) {
      for (int q = 0; q < NW; q++) a.ctl->T[q] = cs[i][q];
      a.ctl->t_found = 1;
    }
  }
}

// Per bucket (one wave): level-1 candidates at or above the threshold.
template <int W>
__global__ __launch_bounds__(64) void k_count_boundary(SelArgs a) {
  constexpr int NW = 1 + 2 * W;
  const uint32_t b = blockIdx.x;
  const uint32_t n = a.cc_in[b];
  uint32_t cnt = 0;
  if (n) {
    uint64_t T[NW];
    for (int q = 0; q < NW; q++) T[q] = a.ctl->T[q];
    const uint32_t ub = a.b_ubase[b];
    const Key<W>* ukb = reinterpret_cast<const Key<W>*>(a.uk);
    for (uint32_t i = threadIdx.x; i < n; i += 64) {
      const uint32_t ui = a.list_in[ub + i];
      uint64_t c[NW];
      composite<W>(a.uc[ui], unmix_key<W>(ukb[ui]), c);
      if (comp_cmp<W>(c, T) >= 0) cnt++;
    }
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_down(cnt, d, 64);
  }
  if (threadIdx.x == 0) a.b_bcnt[b] = cnt;
}

// Output bases: survivors per bucket are counted according to the select
// mode; exclusive scan over the buckets (one block).
enum SelMode : int { S_ALL = 0, S_KEEP_ONLY = 1, S_THRESHOLD = 2 };

__global__ __launch_bounds__(1024) void k_scan_buckets(const uint32_t* b_surv,
                                                       const uint32_t* b_keep,
                                                       const uint32_t* b_abv,
                                                       const uint32_t* b_bcnt, uint32_t nb,
                                                       int sel_mode, uint32_t* b_obase, Ctl* ctl) {
  __shared__ unsigned long long tmp[17];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const uint32_t per = (nb + 1023) / 1024;
  const uint32_t lo = t * per;
  unsigned long long s = 0;
  for (uint32_t k = 0; k < per; k++) {
    const uint32_t b = lo + k;
    if (b < nb) {
      uint32_t c = sel_mode == S_ALL ? b_surv[b]
                   : sel_mode == S_KEEP_ONLY ? b_keep[b]
                                             : b_keep[b] + b_abv[b] + b_bcnt[b];
      s += c;
    }
  }
  unsigned long long x = s;
  for (int d = 1; d < 64; d <<= 1) {
    unsigned long long y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wv] = x;
  __syncthreads();
  if (t == 0) {
    unsigned long long run = 0;
    for (int i = 0; i < 16; i++) {
      unsigned long long q = tmp[i];
      tmp[i] = run;
      run += q;
    }
    tmp[16] = run;
  }
  __syncthreads();
  unsigned long long pre = tmp[wv] + x - s;
  for (uint32_t k = 0; k < per; k++) {
    const uint32_t b = lo + k;
    if (b < nb) {
      b_obase[b] = (uint32_t)pre;
      uint32_t c = sel_mode == S_ALL ? b_surv[b]
                   : sel_mode == S_KEEP_ONLY ? b_keep[b]
                                             : b_keep[b] + b_abv[b] + b_bcnt[b];
      pre += c;
    }
  }
  if (t == 0) ctl->out_total = tmp[16];
}

struct WriteArgs {
  const uint32_t* b_ubase;
  const uint32_t* b_slots;
  const uint32_t* b_obase;
  const void* uk;
  const double2* uc;
  const void* keep_mk;
  int n_keep;
  int sel_mode;
  const Ctl* ctl;
  uint64_t* ox;
  uint64_t* oz;
  void* oc;
  int64_t ocap;
  int out_f32;
};

template <int W>
__global__ __launch_bounds__(256) void k_write(WriteArgs a) {
  constexpr int NW = 1 + 2 * W;
  __shared__ uint32_t scan_tmp[256 / 64 + 1];
  const int tid = threadIdx.x;
  const uint32_t b = blockIdx.x;
  const uint32_t ub = a.b_ubase[b], ns = a.b_slots[b];
  uint32_t obase = a.b_obase[b];
  const Key<W>* uk = reinterpret_cast<const Key<W>*>(a.uk) + ub;
  const double2* uc = a.uc + ub;
  const Key<W>* keep = reinterpret_cast<const Key<W>*>(a.keep_mk);
  uint64_t T[NW];
  if (a.sel_mode == S_THRESHOLD)
    for (int q = 0; q < NW; q++) T[q] = a.ctl->T[q];
  const uint32_t nround = (ns + 255) / 256;
  for (uint32_t r = 0; r < nround; r++) {
    const uint32_t i = r * 256 + tid;
    bool s = false;
    Key<W> raw;
    double2 v = make_double2(0.0, 0.0);
    if (i < ns) {
      v = uc[i];
      if (!is_zero(v)) {
        raw = unmix_key<W>(uk[i]);
        if (a.sel_mode == S_ALL) {
          s = true;
        } else {
          const bool isk = a.n_keep ? keep_lookup<W>(keep, a.n_keep, uk[i]) : false;
          if (isk) s = true;
          else if (a.sel_mode == S_THRESHOLD) {
            uint64_t c[NW];
            composite<W>(v, raw, c);
            s = comp_cmp<W>(c, T) >= 0;
          }
        }
      }
    }
    uint32_t tot;
    const uint32_t pos = block_exclusive_scan(s ? 1u : 0u, scan_tmp, &tot);
    if (s) {
      const size_t o = (size_t)obase + pos;
#pragma unroll
      for (int w = 0; w < W; w++) {
        a.ox[(size_t)w * a.ocap + o] = raw.w[w];
        a.oz[(size_t)w * a.ocap + o] = raw.w[W + w];
      }
      if (a.out_f32) reinterpret_cast<float2*>(a.oc)[o] = make_float2((float)v.x, (float)v.y);
      else reinterpret_cast<double2*>(a.oc)[o] = v;
    }
    obase += tot;
  }
}

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
// H for the commutator emission (one block of 1024 threads, n <= 2047):
// packed raw words [n][2W] in ascending order of lowest site, the index of
// each entry in the caller's H, hstart[s] = first entry with lowest site >= s
// (s = 0 .. 64W + 1; the empty string sorts as site 64W) and the largest
// highest-minus-lowest site.  The order among entries of one lowest site is
// not fixed: every entry carries its own index.
template <int W>
__global__ __launch_bounds__(1024) void k_prep_h(const uint64_t* x, const uint64_t* z, int64_t cap,
                                                 int n, uint64_t* packed, uint32_t* hidx,
                                                 uint32_t* hstart, int* hspan, uint32_t* zero,
                                                 uint32_t nzero) {
  constexpr int SITES = 64 * W;
  __shared__ uint32_t cnt[SITES + 2];
  __shared__ int span;
  const int t = threadIdx.x;
  // also clears `zero` (nzero words: the call's control block)
  for (uint32_t q = t; q < nzero; q += 1024) zero[q] = 0u;
  for (int q = t; q < SITES + 2; q += 1024) cnt[q] = 0u;
  if (t == 0) span = 0;
  __syncthreads();
  int lo[2], rk[2];
  for (int k = 0; k < 2; k++) {
    const int i = t + k * 1024;
    lo[k] = SITES;
    rk[k] = 0;
    if (i < n) {
      int hi = -1;
#pragma unroll
      for (int w = W - 1; w >= 0; w--) {
        const uint64_t s = x[(size_t)w * cap + i] | z[(size_t)w * cap + i];
        if (s) {
          lo[k] = 64 * w + __builtin_ctzll(s);
          if (hi < 0) hi = 64 * w + 63 - __builtin_clzll(s);
        }
      }
      if (hi >= 0) atomicMax(&span, hi - lo[k]);
      rk[k] = (int)atomicAdd(&cnt[lo[k]], 1u);
    }
  }
  __syncthreads();
  if (t == 0) {
    uint32_t run = 0;
    for (int q = 0; q <= SITES; q++) {
      const uint32_t c = cnt[q];
      cnt[q] = run;
      run += c;
    }
    cnt[SITES + 1] = run;
  }
  __syncthreads();
  for (int k = 0; k < 2; k++) {
    const int i = t + k * 1024;
    if (i < n) {
      const int p = (int)cnt[lo[k]] + rk[k];
#pragma unroll
      for (int w = 0; w < W; w++) {
        packed[(size_t)p * 2 * W + w] = x[(size_t)w * cap + i];
        packed[(size_t)p * 2 * W + W + w] = z[(size_t)w * cap + i];
      }
      hidx[p] = (uint32_t)i;
    }
  }
  for (int q = t; q < SITES + 2; q += 1024) hstart[q] = cnt[q];
  if (t == 0) *hspan = span;
}

// Mixed keys of a canonical operator; flags a violation of ascending order.
template <int W>
__global__ void k_mix_keys(const uint64_t* x, const uint64_t* z, int64_t cap, int64_t n,
                           Key<W>* out, unsigned int* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Key<W> raw;
#pragma unroll
  for (int w = 0; w < W; w++) {
    raw.w[w] = x[(size_t)w * cap + i];
    raw.w[W + w] = z[(size_t)w * cap + i];
  }
  const Key<W> m = mix_key<W>(raw);
  out[i] = m;
  if (i > 0) {
    Key<W> rp;
#pragma unroll
    for (int w = 0; w < W; w++) {
      rp.w[w] = x[(size_t)w * cap + i - 1];
      rp.w[W + w] = z[(size_t)w * cap + i - 1];
    }
    if (key_cmp<W>(mix_key<W>(rp), m) >= 0) atomicOr(bad, 1u);
  }
}

// Depolarizing noise in place: c_k *= f[len_k], f[w] = exp(-lambda w)
// computed on the host (len = sites with x or z set).  FP32 coefficients are
// scaled in double and rounded once.
constexpr int NOISE_TABLE = 129;  // lengths 0..128
struct NoiseTable {
  double f[NOISE_TABLE];
};
template <int W>
__global__ __launch_bounds__(256) void k_add_noise(const uint64_t* x, const uint64_t* z,
                                                   int64_t cap, int64_t n, void* coef, int f32,
                                                   NoiseTable t) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    int len = 0;
#pragma unroll
    for (int w = 0; w < W; w++) len += __popcll(x[(size_t)w * cap + i] | z[(size_t)w * cap + i]);
    const double f = t.f[len];
    if (f32) {
      float2* c = reinterpret_cast<float2*>(coef) + i;
      const float2 v = *c;
      *c = make_float2((float)((double)v.x * f), (float)((double)v.y * f));
    } else {
      double2* c = reinterpret_cast<double2*>(coef) + i;
      const double2 v = *c;
      *c = make_double2(v.x * f, v.y * f);
    }
  }
}

// Adjoint in place: the imaginary part of every coefficient changes sign.
__global__ __launch_bounds__(256) void k_conj(void* coef, int64_t n, int f32) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    if (f32) {
      float2* c = reinterpret_cast<float2*>(coef) + i;
      c->y = -c->y;
    } else {
      double2* c = reinterpret_cast<double2*>(coef) + i;
      c->y = -c->y;
    }
  }
}

// Coefficients in A (canonical: ascending order keys `ak`) of the strings of
// Q: out[q] = A's coefficient of Q's string q, or 0 when A lacks it.
template <int W>
__global__ __launch_bounds__(256) void k_lookup(const Key<W>* ak, const void* acoef, int af32,
                                                int64_t na, const uint64_t* qx,
                                                const uint64_t* qz, int64_t qcap, int64_t nq,
                                                double2* out) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= nq) return;
  Key<W> raw;
#pragma unroll
  for (int w = 0; w < W; w++) {
    raw.w[w] = qx[(size_t)w * qcap + q];
    raw.w[W + w] = qz[(size_t)w * qcap + q];
  }
  const Key<W> mk = mix_key<W>(raw);
  int64_t lo = 0, hi = na;
  double2 v = make_double2(0.0, 0.0);
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int c = key_cmp<W>(ak[mid], mk);
    if (c == 0) {
      if (af32) {
        const float2 f = reinterpret_cast<const float2*>(acoef)[mid];
        v = make_double2((double)f.x, (double)f.y);
      } else {
        v = reinterpret_cast<const double2*>(acoef)[mid];
      }
      break;
    }
    if (c < 0) lo = mid + 1;
    else hi = mid;
  }
  out[q] = v;
}

// H = sum_k T_k(H0) listed as T_0(h_0), T_1(h_0), ..., T_{N-1}(h_0), T_0(h_1), ...
// (entry h N + k: h_h translated by k sites); out word-major with capacity
// nH0 N, FP64 coefficients.
template <int W>
__global__ __launch_bounds__(256) void k_ts_expand(const uint64_t* x, const uint64_t* z,
                                                   int64_t cap, const double2* c, int64_t nh,
                                                   int N, uint64_t* ox, uint64_t* oz,
                                                   double2* oc) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = nh * N;
  if (i >= n) return;
  const int64_t h = i / N;
  const int k = (int)(i % N);
  uint64_t vx[W], vz[W], tx[W], tz[W];
#pragma unroll
  for (int w = 0; w < W; w++) {
    vx[w] = x[(size_t)w * cap + h];
    vz[w] = z[(size_t)w * cap + h];
  }
  // translation by k = rotation down by (N - k) mod N
  const int r = k ? N - k : 0;
  ts_rot_down<W>(vx, N, r, tx);
  ts_rot_down<W>(vz, N, r, tz);
#pragma unroll
  for (int w = 0; w < W; w++) {
    ox[(size_t)w * n + i] = tx[w];
    oz[(size_t)w * n + i] = tz[w];
  }
  oc[i] = c[h];
}

// Per-block double-double partials of sum_k stab(s_k) |c_k|^2: the norm of a
// translation-symmetric operator held as representatives, over N (stab =
// translations k in [0, N) that leave the string unchanged).
template <int W, bool F32>
__global__ __launch_bounds__(256) void k_norm_part_ts(const uint64_t* x, const uint64_t* z,
                                                      int64_t cap, const void* coef, int64_t n,
                                                      int N, double2* part) {
  __shared__ double rh[4], rl[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  dd s = dd_zero();
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256) {
    double2 v;
    if (F32) {
      const float2 f = reinterpret_cast<const float2*>(coef)[i];
      v = make_double2(f.x, f.y);
    } else {
      v = reinterpret_cast<const double2*>(coef)[i];
    }
    uint64_t vx[W], vz[W];
#pragma unroll
    for (int w = 0; w < W; w++) {
      vx[w] = x[(size_t)w * cap + i];
      vz[w] = z[(size_t)w * cap + i];
    }
    const int st = ts_stabilizers<W>(vx, vz, N);
    const double w2 = weight2(v);
    for (int r = 0; r < st; r++) s = dd_add(s, w2);
  }
  for (int d = 32; d >= 1; d >>= 1) {
    dd o;
    o.hi = __shfl_down(s.hi, d, 64);
    o.lo = __shfl_down(s.lo, d, 64);
    if (lane < d) s = dd_add(s, o);
  }
  if (lane == 0) {
    rh[wv] = s.hi;
    rl[wv] = s.lo;
  }
  __syncthreads();
  if (tid == 0) {
    dd t = {rh[0], rl[0]};
    for (int w = 1; w < 4; w++) t = dd_add(t, dd{rh[w], rl[w]});
    part[blockIdx.x] = make_double2(t.hi, t.lo);
  }
}

// Order keys of an operator's strings, and the strings of order keys.
template <int W>
__global__ void k_order_keys(const uint64_t* x, const uint64_t* z, int64_t cap, int64_t n,
                             Key<W>* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Key<W> raw;
#pragma unroll
  for (int w = 0; w < W; w++) {
    raw.w[w] = x[(size_t)w * cap + i];
    raw.w[W + w] = z[(size_t)w * cap + i];
  }
  out[i] = mix_key<W>(raw);
}

template <int W>
__global__ void k_from_order_keys(const Key<W>* keys, int64_t n, uint64_t* x, uint64_t* z,
                                  int64_t cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Key<W> raw = unmix_key<W>(keys[i]);
#pragma unroll
  for (int w = 0; w < W; w++) {
    x[(size_t)w * cap + i] = raw.w[w];
    z[(size_t)w * cap + i] = raw.w[W + w];
  }
}

// Partial double-double sums of |c|^2 per block.
template <bool F32>
__global__ __launch_bounds__(256) void k_norm_part(const void* coef, int64_t n, double2* part) {
  __shared__ double rh[4], rl[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  dd s = dd_zero();
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256) {
    double2 v;
    if (F32) {
      const float2 f = reinterpret_cast<const float2*>(coef)[i];
      v = make_double2(f.x, f.y);
    } else {
      v = reinterpret_cast<const double2*>(coef)[i];
    }
    s = dd_add(s, weight2(v));
  }
  for (int d = 32; d >= 1; d >>= 1) {
    dd o;
    o.hi = __shfl_down(s.hi, d, 64);
    o.lo = __shfl_down(s.lo, d, 64);
    if (lane < d) s = dd_add(s, o);
  }
  if (lane == 0) {
    rh[wv] = s.hi;
    rl[wv] = s.lo;
  }
  __syncthreads();
  if (tid == 0) {
    dd t = {rh[0], rl[0]};
    for (int w = 1; w < 4; w++) t = dd_add(t, dd{rh[w], rl[w]});
    part[blockIdx.x] = make_double2(t.hi, t.lo);
  }
}

// Inner product partials: every string of A is looked up in B's mixed keys.
template <int W>
__global__ __launch_bounds__(256) void k_inner_part(const uint64_t* ax, const uint64_t* az,
                                                    int64_t acap, int64_t na, const void* acoef,
                                                    int af32, const Key<W>* bmk, int64_t nb,
                                                    const void* bcoef, int bf32, double2* part_re,
                                                    double2* part_im) {
  __shared__ double rh[2][4], rl[2][4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  dd sr = dd_zero(), si = dd_zero();
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < na; i += (int64_t)gridDim.x * 256) {
    Key<W> raw;
#pragma unroll
    for (int w = 0; w < W; w++) {
      raw.w[w] = ax[(size_t)w * acap + i];
      raw.w[W + w] = az[(size_t)w * acap + i];
    }
    const Key<W> m = mix_key<W>(raw);
    int64_t lo = 0, hi = nb;
    int64_t found = -1;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      const int c = key_cmp<W>(bmk[mid], m);
      if (c == 0) {
        found = mid;
        break;
      }
      if (c < 0) lo = mid + 1;
      else hi = mid;
    }
    if (found >= 0) {
      double2 av, bv;
      if (af32) {
        const float2 f = reinterpret_cast<const float2*>(acoef)[i];
        av = make_double2(f.x, f.y);
      } else av = reinterpret_cast<const double2*>(acoef)[i];
      if (bf32) {
        const float2 f = reinterpret_cast<const float2*>(bcoef)[found];
        bv = make_double2(f.x, f.y);
      } else bv = reinterpret_cast<const double2*>(bcoef)[found];
      const double p1 = av.x * bv.x, p2 = av.y * bv.y, p3 = av.x * bv.y, p4 = av.y * bv.x;
      sr = dd_add(sr, p1);
      sr = dd_add(sr, p2);
      si = dd_add(si, p3);
      si = dd_add(si, -p4);
    }
  }
  for (int d = 32; d >= 1; d >>= 1) {
    dd o;
    o.hi = __shfl_down(sr.hi, d, 64);
    o.lo = __shfl_down(sr.lo, d, 64);
    if (lane < d) sr = dd_add(sr, o);
    o.hi = __shfl_down(si.hi, d, 64);
    o.lo = __shfl_down(si.lo, d, 64);
    if (lane < d) si = dd_add(si, o);
  }
  if (lane == 0) {
    rh[0][wv] = sr.hi;
    rl[0][wv] = sr.lo;
    rh[1][wv] = si.hi;
    rl[1][wv] = si.lo;
  }
  __syncthreads();
  if (tid == 0) {
    dd t0 = {rh[0][0], rl[0][0]}, t1 = {rh[1][0], rl[1][0]};
    for (int w = 1; w < 4; w++) {
      t0 = dd_add(t0, dd{rh[0][w], rl[0][w]});
      t1 = dd_add(t1, dd{rh[1][w], rl[1][w]});
    }
    part_re[blockIdx.x] = make_double2(t0.hi, t0.lo);
    part_im[blockIdx.x] = make_double2(t1.hi, t1.lo);
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace pauli
