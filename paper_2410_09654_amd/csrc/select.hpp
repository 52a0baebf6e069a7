// Top-M selection and output compaction, driven from the device.
//
// After the merge every bucket b holds its surviving strings (length cap and
// coefficient threshold applied; keys as order keys) at U slots
// [b_ubase[b], b_ubase[b] + b_slots[b]), with per-bucket counts of survivors and keep-set survivors and
// a replicated level-0 histogram of |c|^2 (its top 13 bits) over the non-keep survivors.  The
// kernels below decide, without a host round trip, whether a threshold is
// needed (the keep set is always kept and counts toward M; ties are broken by
// ascending key), find it by a two-level radix select over the composite
// ordering key (|c|^2 bits, then the complemented key words), and write the
// kept strings in bucket order.
//
// Flow (one stream, no host synchronisation in between):
//   k_sel_plan  k_sel_pass1  k_sel_pick1  k_sel_narrow  k_sel_finish
//   k_scan_out  k_write_out
// Candidate lists live per bucket in the bucket's own U slot range, so no
// pass appends through a single global counter except the final list of at
// most FINISH_CAP entries.
// The select kernels return at once unless the plan chose S_THRESHOLD.  When
// more than FINISH_CAP candidates share the first two digits (large groups of
// exactly equal |c|), k_sel_pick1 sets ctl->deep, the later kernels stand
// down and the host finishes the call with the multi-level select.
#pragma once
#include "kernels.hpp"

namespace pauli {

constexpr int SEL_CHUNK = 4;       // buckets per 256-thread block (one wave per bucket)

// Bin holding the K-th largest entry of hist[0..nbins) (bins ordered from the
// top): one block of 1024 threads; every thread gets the bin, the rank of the
// K-th entry inside it (1-based) and the bin's count.  K must lie in
// [1, sum(hist)].  tmp: 19 words of shared memory.
DEV void pick_bin(const uint32_t* hist, int nbins, unsigned long long K,
                  unsigned long long* tmp, unsigned int* out_digit,
                  unsigned long long* out_krem, unsigned long long* out_count) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int per = nbins / 1024;  // 2 or 4
  const int hiB = nbins - t * per;
  if (t == 0) {
    tmp[16] = 0ull;
    tmp[17] = 0ull;
    tmp[18] = 0ull;
  }
  unsigned int hv[4] = {0u, 0u, 0u, 0u};
  unsigned long long s = 0;
  for (int q = 1; q <= per; q++) {
    hv[q - 1] = hist[hiB - q];
    s += hv[q - 1];
  }
  unsigned long long x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    unsigned long long y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wv] = x;
  __syncthreads();
  unsigned long long w = lane < 16 ? tmp[lane] : 0ull;
#pragma unroll
  for (int d = 1; d < 16; d <<= 1) {
    unsigned long long y = __shfl_up(w, d, 64);
    if (lane >= d) w += y;
  }
  const unsigned long long before = wv > 0 ? __shfl(w, wv - 1, 64) : 0ull;
  __syncthreads();
  unsigned long long cum = before + x - s;  // entries in the bins above this thread's
  for (int q = 1; q <= per; q++) {
    const unsigned long long h = hv[q - 1];
    if (cum < K && K <= cum + h) {
      tmp[16] = (unsigned long long)(hiB - q);
      tmp[17] = K - cum;
      tmp[18] = h;
    }
    cum += h;
  }
  __syncthreads();
  *out_digit = (unsigned int)tmp[16];
  *out_krem = tmp[17];
  *out_count = tmp[18];
}

struct PlanArgs {
  const uint32_t* b_slots;
  const uint32_t* b_surv;
  const uint32_t* b_keep;
  const uint32_t* b_unique;  // nullable: leave ctl->u_unique as it is
  uint32_t nbk;
  int want_select;
  long long max_strings;
  const uint32_t* hist0;     // HREP replicas of the level-0 |c|^2 histogram (SEL0_BINS each)
  uint32_t* hist1;           // digit-1 histogram replicas, cleared here (nullable)
  unsigned long long* psum;  // [PLAN_PARTS][4] partial counter sums (k_plan_sums)
  uint32_t* h0sum;           // [SEL0_BINS] the level-0 histogram, replicas summed
  Ctl* ctl;
};

// Reductions feeding k_sel_plan, spread over 3 x PLAN_PARTS blocks of 1024
// threads: blocks [0, P) sum the four per-bucket counters over a P-th of the
// buckets each, blocks [P, 2P) sum the HREP replicas of SEL0_BINS / P bins
// of the level-0 histogram each, blocks [2P, 3P) clear a P-th of the digit-1
// replicas.
constexpr int PLAN_PARTS = 16;
static_assert(SEL0_BINS == PLAN_PARTS * 256 && HREP % 4 == 0 &&
                  HREP * SEL_BINS == PLAN_PARTS * 4096,
              "k_plan_sums: 256 level-0 bins and 4096 digit-1 words per block");
__global__ __launch_bounds__(1024) void k_plan_sums(PlanArgs a) {
  __shared__ unsigned long long red[4][16];
  __shared__ uint32_t hr[4][256];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int blk = blockIdx.x;
  if (blk < PLAN_PARTS) {
    const uint32_t chunk = (a.nbk + PLAN_PARTS - 1) / PLAN_PARTS;
    const uint32_t b0 = min(a.nbk, blk * chunk), b1 = min(a.nbk, b0 + chunk);
    unsigned long long v[4] = {0, 0, 0, 0};
    for (uint32_t b = b0 + t; b < b1; b += 1024) {
      v[0] += a.b_slots[b];
      v[1] += a.b_surv[b];
      v[2] += a.b_keep[b];
      if (a.b_unique) v[3] += a.b_unique[b];
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      unsigned long long x = v[q];
      for (int d = 32; d >= 1; d >>= 1) x += __shfl_down(x, d, 64);
      if (lane == 0) red[q][wv] = x;
    }
    __syncthreads();
    if (t < 4) {
      unsigned long long s = 0;
      for (int w = 0; w < 16; w++) s += red[t][w];
      a.psum[blk * 4 + t] = s;
    }
  } else if (blk < 2 * PLAN_PARTS) {
    const int bin = (blk - PLAN_PARTS) * 256 + (t & 255), g = t >> 8;
    uint32_t s = 0;
#pragma unroll
    for (int r = g; r < HREP; r += 4) s += a.hist0[(size_t)r * SEL0_BINS + bin];
    hr[g][t & 255] = s;
    __syncthreads();
    if (t < 256) a.h0sum[bin] = hr[0][t] + hr[1][t] + hr[2][t] + hr[3][t];
  } else if (a.hist1) {
    uint4* z = reinterpret_cast<uint4*>(a.hist1) + (size_t)(blk - 2 * PLAN_PARTS) * 1024;
    z[t] = make_uint4(0u, 0u, 0u, 0u);
  }
}

// Totals of the per-bucket counters, the select mode, and the level-0 bin of
// the threshold (one block of 1024 threads), from the sums of k_plan_sums.
__global__ __launch_bounds__(1024) void k_sel_plan(PlanArgs a) {
  __shared__ unsigned long long tmp[19];
  __shared__ uint32_t hs[SEL0_BINS];
  __shared__ unsigned long long s_K;
  __shared__ int s_mode;
  const int t = threadIdx.x;
  // the level-0 histogram and the counter totals, reduced by k_plan_sums
  constexpr int BPT0 = SEL0_BINS / 1024;
  uint32_t h0[BPT0];
#pragma unroll
  for (int k = 0; k < BPT0; k++) h0[k] = a.h0sum[k * 1024 + t];
  if (t == 0) {
    unsigned long long tot[4] = {0, 0, 0, 0};
    for (int q = 0; q < 4; q++)
      for (int p = 0; p < PLAN_PARTS; p++) tot[q] += a.psum[p * 4 + q];
    a.ctl->u_slots = tot[0];
    a.ctl->surv_total = tot[1];
    a.ctl->keep_total = tot[2];
    if (a.b_unique) a.ctl->u_unique = tot[3];
    const unsigned long long surv = tot[1], fk = tot[2];
    int mode = S_ALL;
    unsigned long long K = 0;
    if (a.want_select) {
      const long long budget = a.max_strings - (long long)fk;
      const unsigned long long nonkeep = surv - fk;
      if (budget <= 0) mode = fk == surv ? S_ALL : S_KEEP_ONLY;
      else if ((unsigned long long)budget >= nonkeep) mode = S_ALL;
      else {
        mode = S_THRESHOLD;
        K = (unsigned long long)budget;
      }
    }
    s_mode = mode;
    s_K = K;
    a.ctl->sel_mode = mode;
  }
#pragma unroll
  for (int k = 0; k < BPT0; k++) hs[k * 1024 + t] = h0[k];
  __syncthreads();
  if (s_mode != S_THRESHOLD) return;
  unsigned int d0;
  unsigned long long krem, cnt;
  pick_bin(hs, SEL0_BINS, s_K, tmp, &d0, &krem, &cnt);
  if (t == 0) {
    a.ctl->sel_d0 = d0;
    a.ctl->sel_K = krem;
    a.ctl->sel_count = cnt;
    a.ctl->fin_level = cnt <= (unsigned long long)FINISH_CAP ? 0u : 1u;
  }
}

struct Sel2Args {
  const uint32_t* b_ubase;
  const uint32_t* b_slots;
  uint32_t* b_abv;
  uint32_t* b_bcnt;
  const void* uk;
  const double2* uc;
  const void* keep_mk;
  int n_keep;
  uint32_t nbk;
  uint32_t* list0;   // level-1 candidates of bucket b at [b_ubase[b], b_ubase[b] + cc0[b])
  uint32_t* cc0;
  uint32_t* listf;   // candidates of the final bin (<= FINISH_CAP) ...
  uint32_t* listfb;  // ... and their buckets
  uint32_t* hist1;   // HREP replicas of the digit-1 histogram
  Ctl* ctl;
};

// Wave-aggregated append: lanes with `take` get consecutive slots of a
// list whose length lives in *counter.  Call with the whole wave.
DEV uint32_t wave_append(bool take, unsigned long long* counter) {
  const uint64_t m = __ballot(take);
  unsigned long long base = 0;
  if (m) {
    if ((threadIdx.x & 63) == 0) base = atomicAdd(counter, (unsigned long long)__popcll(m));
    base = __shfl(base, 0, 64);
  }
  return (uint32_t)base + mbcnt64(m);
}

// Level 1 over all survivors, one wave per bucket: counts per bucket the
// non-keep survivors whose level-0 digit is above the threshold bin, lists
// those inside it and histograms their digit 1 (when the bin is too large to
// finish directly).
template <int W>
__global__ __launch_bounds__(256) void k_sel_pass1(Sel2Args a) {
  constexpr int NW = 1 + 2 * W;
  if (a.ctl->sel_mode != S_THRESHOLD) return;
  const uint32_t D0 = a.ctl->sel_d0;
  const bool lvl1 = a.ctl->fin_level == 1u;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const Key<W>* ukb = reinterpret_cast<const Key<W>*>(a.uk);
  const Key<W>* keep = reinterpret_cast<const Key<W>*>(a.keep_mk);
  uint32_t* hrep = a.hist1 + (size_t)(blockIdx.x % HREP) * SEL_BINS;
  for (int q = 0; q < SEL_CHUNK / 4; q++) {
    const uint32_t b = blockIdx.x * SEL_CHUNK + q * 4 + wv;
    if (b >= a.nbk) break;
    const uint32_t ub = a.b_ubase[b], ns = a.b_slots[b];
    uint32_t abv = 0, nc = 0;
    double2 vn = (uint32_t)lane < ns ? a.uc[ub + lane] : make_double2(0.0, 0.0);
    for (uint32_t i0 = 0; i0 < ns; i0 += 64) {
      const uint32_t i = i0 + lane;
      bool cand = false;
      const double2 v = vn;  // this iteration's value; the next iteration's load is issued now
      if (i + 64 < ns) vn = a.uc[ub + i + 64];
      if (i < ns) {
        if (!is_zero(v)) {
          bool isk = false;
          Key<W> mk;
          if (a.n_keep) {
            mk = ukb[ub + i];
            isk = keep_lookup<W>(keep, a.n_keep, mk);
          }
          if (!isk) {
            const uint32_t d0 = (uint32_t)((uint64_t)__double_as_longlong(weight2(v)) >> SEL0_SHIFT);
            if (d0 > D0) {
              abv++;
            } else if (d0 == D0) {
              cand = true;
              if (lvl1) {
                // digit 1: the 12 bits of |c|^2 after the level-0 bits (the
                // string words of the composite do not reach it)
                uint64_t c[NW] = {};
                c[0] = (uint64_t)__double_as_longlong(weight2(v));
                atomicAdd(&hrep[comp_digit<W>(c, 1)], 1u);
              }
            }
          }
        }
      }
      const uint64_t m = __ballot(cand);
      if (cand) a.list0[ub + nc + mbcnt64(m)] = ub + i;
      nc += (uint32_t)__popcll(m);
    }
    for (int d = 32; d >= 1; d >>= 1) abv += __shfl_down(abv, d, 64);
    if (lane == 0) {
      a.b_abv[b] = abv;
      a.cc0[b] = nc;
    }
  }
}

// Digit-1 bin of the threshold (one block), from the HREP histogram replicas.
__global__ __launch_bounds__(1024) void k_sel_pick1(const uint32_t* hist1, Ctl* ctl) {
  __shared__ unsigned long long tmp[19];
  __shared__ uint32_t hs[SEL_BINS];
  if (ctl->sel_mode != S_THRESHOLD || ctl->fin_level != 1u) return;
  const unsigned long long K = ctl->sel_K;
  // every load of the replicas issued before the first use
  constexpr int BPT = SEL_BINS / 1024;
  uint32_t h[BPT];
#pragma unroll
  for (int k = 0; k < BPT; k++) {
    h[k] = 0;
#pragma unroll
    for (int r = 0; r < HREP; r++) h[k] += hist1[(size_t)r * SEL_BINS + k * 1024 + threadIdx.x];
  }
#pragma unroll
  for (int k = 0; k < BPT; k++) hs[k * 1024 + threadIdx.x] = h[k];
  __syncthreads();
  unsigned int d1;
  unsigned long long krem, cnt;
  pick_bin(hs, SEL_BINS, K, tmp, &d1, &krem, &cnt);
  if (threadIdx.x == 0) {
    ctl->sel_d1 = d1;
    ctl->sel_K = krem;
    ctl->sel_count = cnt;
    if (cnt > (unsigned long long)FINISH_CAP) ctl->deep = 1u;
  }
}

// The final candidates, gathered into one list: the level-1 candidates
// inside the digit-1 bin, or all of them when the level-0 bin is small.
// Also counts per bucket the candidates above the digit-1 bin.  One wave per
// bucket.
template <int W>
__global__ __launch_bounds__(256) void k_sel_narrow(Sel2Args a) {
  constexpr int NW = 1 + 2 * W;
  if (a.ctl->sel_mode != S_THRESHOLD || a.ctl->deep) return;
  const bool l1 = a.ctl->fin_level == 1u;
  const uint32_t D1 = a.ctl->sel_d1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int q = 0; q < SEL_CHUNK / 4; q++) {
    const uint32_t b = blockIdx.x * SEL_CHUNK + q * 4 + wv;
    if (b >= a.nbk) break;
    const uint32_t ub = a.b_ubase[b], n = a.cc0[b];
    uint32_t above = 0;
    for (uint32_t i0 = 0; i0 < n; i0 += 64) {
      const uint32_t i = i0 + lane;
      bool take = false;
      uint32_t ui = 0;
      if (i < n) {
        ui = a.list0[ub + i];
        take = true;
        if (l1) {
          // the digit-1 bin holds the 12 bits of |c|^2 after the level-0 bits:
          // the string words of the composite do not reach it
          uint64_t c[NW] = {};
          c[0] = (uint64_t)__double_as_longlong(weight2(a.uc[ui]));
          const uint32_t d1 = comp_digit<W>(c, 1);
          take = d1 == D1;
          above += d1 > D1 ? 1u : 0u;
        }
      }
      const uint32_t pos = wave_append(take, &a.ctl->cand_n[1]);
      if (take && pos < (uint32_t)FINISH_CAP) {
        a.listf[pos] = ui;
        a.listfb[pos] = b;
      }
    }
    // candidates above the final bin are above the threshold; k_sel_finish
    // adds those of the final bin at or above it
    for (int d = 32; d >= 1; d >>= 1) above += __shfl_down(above, d, 64);
    if (lane == 0) a.b_bcnt[b] = above;
  }
}

// Threshold: the K-th largest composite among the final candidates (one
// block; bitonic sort, descending, of the next power of two >= their number
// in LDS).  The K entries at or above it are counted into their buckets.
template <int W>
__global__ __launch_bounds__(1024) void k_sel_finish(Sel2Args a) {
  constexpr int NW = 1 + 2 * W;
  static_assert(FINISH_CAP == 2048, "bitonic sort of up to 2048 entries with 1024 threads");
  __shared__ uint64_t cs[FINISH_CAP][NW];
  __shared__ uint32_t cb[FINISH_CAP];
  if (a.ctl->sel_mode != S_THRESHOLD || a.ctl->deep) return;
  const unsigned long long n = a.ctl->cand_n[1];
  const unsigned long long K = a.ctl->sel_K;
  if (n > (unsigned long long)FINISH_CAP || K < 1 || K > n) {
    if (threadIdx.x == 0) a.ctl->deep = 1u;
    return;
  }
  int P = 2;
  while ((unsigned long long)P < n) P <<= 1;
  const Key<W>* ukb = reinterpret_cast<const Key<W>*>(a.uk);
  const int t = threadIdx.x;
  for (int i = t; i < P; i += 1024) {
    uint64_t c[NW];
    uint32_t bk = 0;
    if ((unsigned long long)i < n) {
      const uint32_t ui = a.listf[i];
      bk = a.listfb[i];
      composite<W>(a.uc[ui], unmix_key<W>(ukb[ui]), c);
    } else {
#pragma unroll
      for (int q = 0; q < NW; q++) c[q] = 0ull;  // below every entry
    }
#pragma unroll
    for (int q = 0; q < NW; q++) cs[i][q] = c[q];
    cb[i] = bk;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (t < (P >> 1)) {
        const int i = 2 * t - (t & (j - 1));
        const int l = i + j;
        uint64_t x[NW], y[NW];
#pragma unroll
        for (int q = 0; q < NW; q++) {
          x[q] = cs[i][q];
          y[q] = cs[l][q];
        }
        // x < y, lexicographic, without branches
        bool lt = false;
#pragma unroll
        for (int q = NW - 1; q >= 0; q--) lt = (x[q] < y[q]) | ((x[q] == y[q]) & lt);
        bool gt = false;
#pragma unroll
        for (int q = NW - 1; q >= 0; q--) gt = (x[q] > y[q]) | ((x[q] == y[q]) & gt);
        const bool desc = (i & k) == 0;
        if (desc ? lt : gt) {
#pragma unroll
          for (int q = 0; q < NW; q++) {
            cs[i][q] = y[q];
            cs[l][q] = x[q];
          }
          const uint32_t tb = cb[i];
          cb[i] = cb[l];
          cb[l] = tb;
        }
      }
      __syncthreads();
    }
  }
  for (int i = t; (unsigned long long)i < K; i += 1024) atomicAdd(&a.b_bcnt[cb[i]], 1u);
  if (t == 0) {
#pragma unroll
    for (int q = 0; q < NW; q++) a.ctl->T[q] = cs[K - 1][q];
    a.ctl->t_found = 1u;
  }
}

// Eight consecutive words p[b0 .. b0 + 8) (zero past nb), as two 16-byte
// loads when the eight lie inside the array (b0 is a multiple of 8 and the
// arena aligns the tables to 256 bytes).
DEV void load8(const uint32_t* p, uint32_t b0, uint32_t nb, uint32_t* v) {
  if (b0 + 8 <= nb) {
    const uint4 a = *reinterpret_cast<const uint4*>(p + b0);
    const uint4 c = *reinterpret_cast<const uint4*>(p + b0 + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = c.x; v[5] = c.y; v[6] = c.z; v[7] = c.w;
  } else {
#pragma unroll
    for (int k = 0; k < 8; k++) v[k] = b0 + k < nb ? p[b0 + k] : 0u;
  }
}

// Output bases: survivors kept per bucket (by the select mode), exclusive
// scan over the buckets in tiles of 8192 (one block; thread t owns eight
// consecutive buckets, read and written as 16-byte vectors).
__global__ __launch_bounds__(1024) void k_scan_out(const uint32_t* b_surv, const uint32_t* b_keep,
                                                   const uint32_t* b_abv, const uint32_t* b_bcnt,
                                                   uint32_t nb, uint32_t* b_obase, Ctl* ctl) {
  constexpr int PER = 8, TILE = 1024 * PER;
  __shared__ unsigned long long tmp[17];
  if (ctl->deep) return;
  const int mode = ctl->sel_mode;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  unsigned long long carry = 0;
  for (uint32_t base = 0; base < nb; base += TILE) {
    const uint32_t b0 = base + (uint32_t)t * PER;
    uint32_t loc[PER];
    if (mode == S_ALL) {
      load8(b_surv, b0, nb, loc);
    } else if (mode == S_KEEP_ONLY) {
      load8(b_keep, b0, nb, loc);
    } else {
      uint32_t a[PER], c[PER];
      load8(b_keep, b0, nb, loc);
      load8(b_abv, b0, nb, a);
      load8(b_bcnt, b0, nb, c);
#pragma unroll
      for (int k = 0; k < PER; k++) loc[k] += a[k] + c[k];
    }
    unsigned long long s = 0;
#pragma unroll
    for (int k = 0; k < PER; k++) s += loc[k];
    unsigned long long x = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      unsigned long long y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) tmp[wv] = x;
    __syncthreads();
    unsigned long long w = lane < 16 ? tmp[lane] : 0ull;
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
      unsigned long long y = __shfl_up(w, d, 64);
      if (lane >= d) w += y;
    }
    const unsigned long long before = wv > 0 ? __shfl(w, wv - 1, 64) : 0ull;
    const unsigned long long tile_total = __shfl(w, 15, 64);
    unsigned long long pre = carry + before + x - s;
    uint32_t o[PER];
#pragma unroll
    for (int k = 0; k < PER; k++) {
      o[k] = (uint32_t)pre;
      pre += loc[k];
    }
    if (b0 + PER <= nb) {
      *reinterpret_cast<uint4*>(b_obase + b0) = make_uint4(o[0], o[1], o[2], o[3]);
      *reinterpret_cast<uint4*>(b_obase + b0 + 4) = make_uint4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
      for (int k = 0; k < PER; k++)
        if (b0 + k < nb) b_obase[b0 + k] = o[k];
    }
    carry += tile_total;
    __syncthreads();  // tmp is rewritten by the next tile
  }
  if (t == 0) ctl->out_total = carry;
}

// Kept strings in bucket order, one wave per bucket.  Writes nothing when the
// output does not fit (the host reports the size).
template <int W>
__global__ __launch_bounds__(256) void k_write_out(WriteArgs a, uint32_t nbk) {
  constexpr int NW = 1 + 2 * W;
  if (a.ctl->deep || a.ctl->out_total > (unsigned long long)a.ocap) return;
  const int mode = a.ctl->sel_mode;
  uint64_t T[NW];
  if (mode == S_THRESHOLD)
#pragma unroll
    for (int q = 0; q < NW; q++) T[q] = a.ctl->T[q];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const Key<W>* ukb = reinterpret_cast<const Key<W>*>(a.uk);
  const Key<W>* keep = reinterpret_cast<const Key<W>*>(a.keep_mk);
  for (int q = 0; q < SEL_CHUNK / 4; q++) {
    const uint32_t b = blockIdx.x * SEL_CHUNK + q * 4 + wv;
    if (b >= nbk) break;
    const uint32_t ub = a.b_ubase[b], ns = a.b_slots[b];
    uint32_t obase = a.b_obase[b];
    double2 vn = (uint32_t)lane < ns ? a.uc[ub + lane] : make_double2(0.0, 0.0);
    for (uint32_t i0 = 0; i0 < ns; i0 += 64) {
      const uint32_t i = i0 + lane;
      bool s = false, have_raw = false;
      Key<W> raw;
      const double2 v = vn;  // this iteration's value; the next iteration's load is issued now
      if (i + 64 < ns) vn = a.uc[ub + i + 64];
      if (i < ns) {
        if (!is_zero(v)) {
          if (mode == S_ALL) {
            s = true;
          } else {
            bool isk = false;
            if (a.n_keep) isk = keep_lookup<W>(keep, a.n_keep, ukb[ub + i]);
            if (isk) {
              s = true;
            } else if (mode == S_THRESHOLD) {
              // |c|^2 bits decide unless they equal the threshold's
              const uint64_t m2 = (uint64_t)__double_as_longlong(weight2(v));
              if (m2 != T[0]) {
                s = m2 > T[0];
              } else {
                raw = unmix_key<W>(ukb[ub + i]);
                have_raw = true;
                uint64_t c[NW];
                composite<W>(v, raw, c);
                s = comp_cmp<W>(c, T) >= 0;
              }
            }
          }
        }
      }
      const uint64_t m = __ballot(s);
      if (s) {
        if (!have_raw) raw = unmix_key<W>(ukb[ub + i]);
        const size_t o = (size_t)obase + mbcnt64(m);
#pragma unroll
        for (int w = 0; w < W; w++) {
          a.ox[(size_t)w * a.ocap + o] = raw.w[w];
          a.oz[(size_t)w * a.ocap + o] = raw.w[W + w];
        }
        if (a.out_f32) reinterpret_cast<float2*>(a.oc)[o] = make_float2((float)v.x, (float)v.y);
        else reinterpret_cast<double2*>(a.oc)[o] = v;
      }
      obase += (uint32_t)__popcll(m);
    }
  }
}

}  // namespace pauli
