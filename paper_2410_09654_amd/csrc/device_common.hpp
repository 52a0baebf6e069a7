// Device-side helpers of the Pauli-string engine (gfx950, wave64).
//
// Key words: a string on W 64-bit words per mask is kept as 2W words,
// raw order (x[0..W-1], z[0..W-1]).  Inside the engine strings travel as
// "mixed keys": a two-round Feistel network over the two halves (x, z)
// whose round function is built from the MurmurHash3 64-bit finalizer
// (fmix64).  The mix is a bijection, so equal mixed keys mean equal strings,
// its leading bits are uniformly spread (they choose the hash bins), and the
// ascending order of mixed keys is the library's canonical storage order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DEV __device__ __forceinline__

namespace pauli {

constexpr int NBINS_LOG = 14;
constexpr int NBINS = 1 << NBINS_LOG;   // hash bins of a call that fits one pass
constexpr int NBINS_LOG_SMALL = 10;     // hash bins of a call of at most 2^18 records
constexpr int NBINS_LOG_MP = 15;        // hash bins per pass of a call that needs
constexpr int NBINS_MP = 1 << NBINS_LOG_MP;  // several (twice the records per pass)
constexpr int MERGE_CAP = 1984;         // max records of one merge bucket (LDS: two
                                        // merge blocks per CU at W = 1)
// The bucket capacity per key width: two merge blocks per CU in LDS at
// W = 2 too (52 bytes per record in FP64).
template <int W>
constexpr int merge_cap() { return W == 1 ? MERGE_CAP : 1344; }
constexpr int MERGE_THREADS = 1024;   // 16 waves; two merge blocks per CU (8 waves/SIMD)
// Small-bucket merge: 512 threads and an LDS footprint of at most 53 KiB
// (keys, values and source ids per record plus the 8 KiB digit table), so
// three blocks share a CU; larger buckets go to the full-size merge.
constexpr int MERGE_SMALL_THREADS = 512;
template <int W, bool F32>
constexpr int small_merge_cap() {
  return ((53 * 1024 - 9 * 1024) / (16 * W + (F32 ? 8 : 16) + 4)) & ~63;
}
constexpr int DIGIT_BITS = 11;          // in-bucket counting-sort digit
constexpr int NDIGITS = 1 << DIGIT_BITS;
constexpr int EMIT_THREADS = 1024;
constexpr int SEL0_SHIFT = 51;          // level-0 select bin of |c|^2: its bits >> 51
constexpr int SEL0_BINS = 4096;         // (exponent and first mantissa bit; |c|^2 >= 0)
constexpr int SEL_BINS = 4096;          // 12-bit digits of later select levels
constexpr int FINISH_CAP = 2048;
constexpr int HREP = 16;                // replicas of the select histograms
                                        // (blocks add into replica blockIdx % HREP)
constexpr uint32_t GROUP_SHIFT = 28;    // record source id = group << 28 | index

constexpr uint64_t MIX_C1 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t MIX_C2 = 0xC2B2AE3D27D4EB4Full;

DEV uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

template <int W>
struct Key {
  uint64_t w[2 * W];
};

// Feistel round function of one half (W words) -> W words.
template <int W>
DEV void mix_round(const uint64_t* in, uint64_t* out, uint64_t c) {
  if constexpr (W == 1) {
    out[0] = fmix64(in[0] ^ c);
  } else {
    uint64_t s = fmix64(in[0] ^ c);
    s = fmix64(s ^ in[1]);
    out[0] = s;
    out[1] = fmix64(s ^ c ^ 0x5bd1e9955bd1e995ull);
  }
}

template <int W>
DEV Key<W> mix_key(const Key<W>& raw) {
  uint64_t L[W], R[W], f[W];
#pragma unroll
  for (int i = 0; i < W; i++) {
    L[i] = raw.w[i];
    R[i] = raw.w[W + i];
  }
  mix_round<W>(L, f, MIX_C1);
#pragma unroll
  for (int i = 0; i < W; i++) R[i] ^= f[i];
  mix_round<W>(R, f, MIX_C2);
#pragma unroll
  for (int i = 0; i < W; i++) L[i] ^= f[i];
  Key<W> m;
#pragma unroll
  for (int i = 0; i < W; i++) {
    m.w[i] = L[i];
    m.w[W + i] = R[i];
  }
  return m;
}

template <int W>
DEV Key<W> unmix_key(const Key<W>& m) {
  uint64_t L[W], R[W], f[W];
#pragma unroll
  for (int i = 0; i < W; i++) {
    L[i] = m.w[i];
    R[i] = m.w[W + i];
  }
  mix_round<W>(R, f, MIX_C2);
#pragma unroll
  for (int i = 0; i < W; i++) L[i] ^= f[i];
  mix_round<W>(L, f, MIX_C1);
#pragma unroll
  for (int i = 0; i < W; i++) R[i] ^= f[i];
  Key<W> raw;
#pragma unroll
  for (int i = 0; i < W; i++) {
    raw.w[i] = L[i];
    raw.w[W + i] = R[i];
  }
  return raw;
}

// -1 / 0 / 1 lexicographic comparison, word 0 most significant.
template <int W>
DEV int key_cmp(const Key<W>& a, const Key<W>& b) {
  // lexicographic over the words, written without branches (the word
  // comparisons are combined with bitwise operators)
  bool lt = false, gt = false;
#pragma unroll
  for (int i = 2 * W - 1; i >= 0; i--) {
    const bool eq = a.w[i] == b.w[i];
    lt = (a.w[i] < b.w[i]) | (eq & lt);
    gt = (a.w[i] > b.w[i]) | (eq & gt);
  }
  return (int)gt - (int)lt;
}

// (a, xa) < (b, xb) in (key, source id) order, without branches.
template <int W>
DEV bool key_src_less(const Key<W>& a, uint32_t xa, const Key<W>& b, uint32_t xb) {
  bool lt = xa < xb;
#pragma unroll
  for (int i = 2 * W - 1; i >= 0; i--) lt = (a.w[i] < b.w[i]) | ((a.w[i] == b.w[i]) & lt);
  return lt;
}

template <int W>
DEV bool key_eq(const Key<W>& a, const Key<W>& b) {
  bool e = true;
#pragma unroll
  for (int i = 0; i < 2 * W; i++) e = e & (a.w[i] == b.w[i]);
  return e;
}

// ---------------------------------------------------------------------------
// Translation-symmetric operators on a periodic chain of N sites (site j is
// bit j of the W words, bits from N up are zero).  T_k moves site j to site
// (j + k) mod N.  The orbit representative is the rotation whose occupied
// pattern x|z, read as an N-bit number, is smallest; ties by x, then z.
// ---------------------------------------------------------------------------
// v rotated so that site j of the result is site (j + r) mod N of v (0 <= r < N).
template <int W>
DEV void ts_rot_down(const uint64_t* v, int N, int r, uint64_t* out) {
  if constexpr (W == 1) {
    const uint64_t m = N == 64 ? ~0ull : ((1ull << N) - 1ull);
    out[0] = r ? (((v[0] >> r) | (v[0] << (N - r))) & m) : v[0];
  } else {
    // 128-bit: lo = v[0], hi = v[1]
    auto shr = [](uint64_t lo, uint64_t hi, int s, uint64_t& olo, uint64_t& ohi) {
      if (s == 0) { olo = lo; ohi = hi; }
      else if (s < 64) { olo = (lo >> s) | (hi << (64 - s)); ohi = hi >> s; }
      else { olo = hi >> (s - 64); ohi = 0; }
    };
    auto shl = [](uint64_t lo, uint64_t hi, int s, uint64_t& olo, uint64_t& ohi) {
      if (s == 0) { olo = lo; ohi = hi; }
      else if (s < 64) { ohi = (hi << s) | (lo >> (64 - s)); olo = lo << s; }
      else { ohi = lo << (s - 64); olo = 0; }
    };
    if (r == 0) {
      out[0] = v[0];
      out[1] = v[1];
      return;
    }
    uint64_t alo, ahi, blo, bhi;
    shr(v[0], v[1], r, alo, ahi);
    shl(v[0], v[1], N - r, blo, bhi);
    uint64_t lo = alo | blo, hi = ahi | bhi;
    if (N <= 64) {
      lo &= N == 64 ? ~0ull : ((1ull << N) - 1ull);
      hi = 0;
    } else if (N < 128) {
      hi &= (1ull << (N - 64)) - 1ull;
    }
    out[0] = lo;
    out[1] = hi;
  }
}

// -1 / 0 / 1 comparison of W-word numbers, word W-1 most significant.
template <int W>
DEV int num_cmp(const uint64_t* a, const uint64_t* b) {
  int c = 0;
#pragma unroll
  for (int i = 0; i < W; i++) c = a[i] != b[i] ? (a[i] < b[i] ? -1 : 1) : c;
  return c;
}

// Translations T_r, r in [0, N), that leave the string (x, z) unchanged:
// N / p for the string's period p (the smallest divisor r of N with T_r s = s).
template <int W>
DEV int ts_stabilizers(const uint64_t* x, const uint64_t* z, int N) {
  for (int r = 1; r < N; r++) {
    if (N % r) continue;
    uint64_t tx[W], tz[W];
    ts_rot_down<W>(x, N, r, tx);
    ts_rot_down<W>(z, N, r, tz);
    if (num_cmp<W>(tx, x) == 0 && num_cmp<W>(tz, z) == 0) return N / r;
  }
  return 1;
}

// Occupied sites r (bit r of the result) that end a longest cyclic run of
// empty sites, i.e. the rotations r (site r moved to site 0) whose occupied
// pattern has the most leading zeros as an N-bit number: the only rotations
// that can be smallest.  One-word strings (N <= 64) with at least one empty
// site.  Bit s of A[j]: sites s, ..., s + 2^j - 1 (mod N) all empty; the
// longest run G is then found by doubling and halving, and the runs of
// length G that start at the set bits of `cur` end below sites s + G.
DEV uint64_t ts_gap_candidates(uint64_t m, int N) {
  const uint64_t mask = N == 64 ? ~0ull : ((1ull << N) - 1ull);
  const uint64_t e = ~m & mask;
  uint64_t A[6];
  A[0] = e;
  int lev = 0;
#pragma unroll
  for (int j = 1; j < 6; j++) {
    if ((1 << (j - 1)) >= N) break;
    uint64_t r;
    ts_rot_down<1>(&A[j - 1], N, 1 << (j - 1), &r);
    A[j] = A[j - 1] & r;
    if (!A[j]) break;
    lev = j;
  }
  uint64_t cur = A[lev];
  int G = 1 << lev;  // a run of G empty sites starts at each set bit of cur; G < N
#pragma unroll
  for (int j = 4; j >= 0; j--) {
    if (j >= lev) continue;
    uint64_t r;
    ts_rot_down<1>(&A[j], N, G, &r);
    const uint64_t t = cur & r;
    if (t) {
      cur = t;
      G += 1 << j;
    }
  }
  uint64_t c;
  ts_rot_down<1>(&cur, N, N - G, &c);  // bit s + G for every start s
  return c;
}

// The orbit representative of the raw key k (x words, then z words), in place;
// returns the rotation r (site r moved to site 0), the smallest one when
// several give the representative.  Only rotations that bring an occupied
// site to site 0 can be smallest, and of those (one-word strings with more
// than a few occupied sites) only the ones after a longest empty run.
template <int W>
DEV int ts_representative(uint64_t* k, int N) {
  int best = -1;
  uint64_t m[W], cand[W], bm[W], bx[W], bz[W];
#pragma unroll
  for (int i = 0; i < W; i++) {
    m[i] = k[i] | k[W + i];
    cand[i] = m[i];
    bm[i] = m[i];
    bx[i] = k[i];
    bz[i] = k[W + i];
  }
  if constexpr (W == 1) {
    const int p = __popcll(m[0]);
    if (p > 6 && p < N) cand[0] = ts_gap_candidates(m[0], N);
  }
#pragma unroll
  for (int w = 0; w < W; w++) {
    uint64_t bits = cand[w];
    while (bits) {
      const int r = 64 * w + __builtin_ctzll(bits);
      bits &= bits - 1;
      uint64_t tm[W], tx[W], tz[W];
      ts_rot_down<W>(m, N, r, tm);
      ts_rot_down<W>(k, N, r, tx);
      ts_rot_down<W>(k + W, N, r, tz);
      int c = -1;
      if (best >= 0) {
        c = num_cmp<W>(tm, bm);
        if (c == 0) c = num_cmp<W>(tx, bx);
        if (c == 0) c = num_cmp<W>(tz, bz);
      }
      if (c < 0) {
        best = r;
#pragma unroll
        for (int i = 0; i < W; i++) {
          bm[i] = tm[i];
          bx[i] = tx[i];
          bz[i] = tz[i];
        }
      }
    }
  }
  if (best < 0) return 0;  // the identity string
#pragma unroll
  for (int i = 0; i < W; i++) {
    k[i] = bx[i];
    k[W + i] = bz[i];
  }
  return best;
}

// Number of non-identity sites of a raw key.
template <int W>
DEV int key_length(const Key<W>& raw) {
  int n = 0;
#pragma unroll
  for (int i = 0; i < W; i++) n += __popcll(raw.w[i] | raw.w[W + i]);
  return n;
}

// ---------------------------------------------------------------------------
// Complex arithmetic, no contraction (the library is compiled with
// -ffp-contract=off): (ar br - ai bi, ar bi + ai br), each product rounded.
// ---------------------------------------------------------------------------
DEV double2 cmul(double2 a, double2 b) {
  double p1 = a.x * b.x, p2 = a.y * b.y, p3 = a.x * b.y, p4 = a.y * b.x;
  return make_double2(p1 - p2, p3 + p4);
}
DEV float2 cmulf(float2 a, float2 b) {
  float p1 = a.x * b.x, p2 = a.y * b.y, p3 = a.x * b.y, p4 = a.y * b.x;
  return make_float2(p1 - p2, p3 + p4);
}
// 2 i^e v, exact.
DEV double2 times_2ie(double2 v, int e) {
  double2 r;
  switch (e & 3) {
    case 0: r = make_double2(2.0 * v.x, 2.0 * v.y); break;
    case 1: r = make_double2(-2.0 * v.y, 2.0 * v.x); break;
    case 2: r = make_double2(-2.0 * v.x, -2.0 * v.y); break;
    default: r = make_double2(2.0 * v.y, -2.0 * v.x); break;
  }
  return r;
}
DEV float2 times_2ie(float2 v, int e) {
  float2 r;
  switch (e & 3) {
    case 0: r = make_float2(2.0f * v.x, 2.0f * v.y); break;
    case 1: r = make_float2(-2.0f * v.y, 2.0f * v.x); break;
    case 2: r = make_float2(-2.0f * v.x, -2.0f * v.y); break;
    default: r = make_float2(2.0f * v.y, -2.0f * v.x); break;
  }
  return r;
}
// i^e v, exact.
DEV double2 times_ie(double2 v, int e) {
  double2 r;
  switch (e & 3) {
    case 0: r = v; break;
    case 1: r = make_double2(-v.y, v.x); break;
    case 2: r = make_double2(-v.x, -v.y); break;
    default: r = make_double2(v.y, -v.x); break;
  }
  return r;
}
DEV float2 times_ie(float2 v, int e) {
  float2 r;
  switch (e & 3) {
    case 0: r = v; break;
    case 1: r = make_float2(-v.y, v.x); break;
    case 2: r = make_float2(-v.x, -v.y); break;
    default: r = make_float2(v.y, -v.x); break;
  }
  return r;
}
DEV double weight2(double2 v) {
  double a = v.x * v.x;
  double b = v.y * v.y;
  return a + b;
}
DEV bool is_zero(double2 v) { return v.x == 0.0 && v.y == 0.0; }

// Kahan-compensated accumulation (one component).
DEV void kahan_add(float& s, float& comp, float t) {
  float y = t - comp;
  float u = s + y;
  comp = (u - s) - y;
  s = u;
}

// ---------------------------------------------------------------------------
// Double-double accumulation of non-negative or signed terms.
// ---------------------------------------------------------------------------
struct dd {
  double hi, lo;
};
DEV dd dd_zero() { return {0.0, 0.0}; }
DEV void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
DEV dd dd_add(dd a, double b) {
  double s, e;
  two_sum(a.hi, b, s, e);
  e = e + a.lo;
  double hi = s + e;
  double lo = e - (hi - s);
  return {hi, lo};
}
DEV dd dd_add(dd a, dd b) {
  double s, e;
  two_sum(a.hi, b.hi, s, e);
  e = e + (a.lo + b.lo);
  double hi = s + e;
  double lo = e - (hi - s);
  return {hi, lo};
}

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------
DEV uint32_t lane_id() { return __lane_id(); }
DEV uint32_t mbcnt64(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block-wide exclusive scan of one uint32 per thread (blockDim <= 1024).
// `tmp` must hold blockDim.x/64 + 1 words.  Returns the exclusive prefix and
// writes the total into *total.
DEV uint32_t block_exclusive_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wv] = x;
  __syncthreads();
  // every wave scans the (at most 16) wave totals itself
  uint32_t t = lane < nw ? tmp[lane] : 0u;
#pragma unroll
  for (int d = 1; d < 16; d <<= 1) {
    uint32_t y = __shfl_up(t, d, 64);
    if (lane >= d) t += y;
  }
  const uint32_t before = wv > 0 ? __shfl(t, wv - 1, 64) : 0u;
  *total = __shfl(t, nw - 1, 64);
  __syncthreads();  // tmp may be reused by the next scan
  return before + x - v;
}

}  // namespace pauli
