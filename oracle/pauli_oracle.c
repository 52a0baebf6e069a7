/* Plain CPU oracle for the Pauli-string operator algebra.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Slow on purpose
 * and written to be checked against the paper by eye:
 *   - string products go site by site through the textbook table of
 *     single-site Pauli products (Methods, "Pauli strings"), not through the
 *     popcount formulas the GPU path uses;
 *   - the commutator follows Alg. 1 in commutator form: every (H string,
 *     O string) pair, with the coefficient (phi_ab - phi_ba) h_a c_b, summed
 *     per output string in ascending H index (a dictionary is replaced by
 *     sorting the records by (key, H index) and folding each run in order);
 *   - truncation keeps strings of length <= L, |c| >= eps, then the M largest
 *     |c| (ties: smaller key first) with the keep set always retained
 *     (trim/cutoff of the Methods section and of the Lanczos listing);
 *   - norms and inner products are exact sums rounded once (a fixed-point
 *     accumulator wide enough for every double).
 * Floating point: compiled with -ffp-contract=off; complex products are
 * (fl(ar*br) - fl(ai*bi), fl(ar*bi) + fl(ai*br)).
 */
#include "pauli_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Single-site Pauli algebra.  Site code = xbit + 2*zbit: I=0 X=1 Z=2 Y=3.  */
/* Row = left factor, column = right factor, both in the order I, X, Z, Y.  */
/* P_row P_col = i^K P_R.                                                    */
/* ------------------------------------------------------------------------ */
static const char SITE_NAME[4] = {'I', 'X', 'Z', 'Y'};
static const char MUL_R[4][4] = {
    /*        I    X    Z    Y  */
    /* I */ {'I', 'X', 'Z', 'Y'},
    /* X */ {'X', 'I', 'Y', 'Z'},
    /* Z */ {'Z', 'Y', 'I', 'X'},
    /* Y */ {'Y', 'Z', 'X', 'I'},
};
static const int MUL_K[4][4] = {
    /*        I  X  Z  Y  */
    /* I */ {0, 0, 0, 0},
    /* X */ {0, 0, 3, 1}, /* XZ = -iY, XY = iZ */
    /* Z */ {0, 1, 0, 3}, /* ZX = iY,  ZY = -iX */
    /* Y */ {0, 3, 1, 0}, /* YX = -iZ, YZ = iX */
};

static int code_of_name(char c) {
  for (int k = 0; k < 4; k++)
    if (SITE_NAME[k] == c) return k;
  return -1;
}

static int site_code(const uint64_t x[2], const uint64_t z[2], int j) {
  int w = j / 64, b = j % 64;
  return (int)((x[w] >> b) & 1u) + 2 * (int)((z[w] >> b) & 1u);
}

static void set_site(uint64_t x[2], uint64_t z[2], int j, int code) {
  int w = j / 64, b = j % 64;
  if (code & 1) x[w] |= (uint64_t)1 << b;
  if (code & 2) z[w] |= (uint64_t)1 << b;
}

void or_string_product(int n_qubits, const uint64_t ax[2], const uint64_t az[2],
                       const uint64_t bx[2], const uint64_t bz[2], uint64_t cx[2],
                       uint64_t cz[2], int *k) {
  int phase = 0;
  cx[0] = cx[1] = cz[0] = cz[1] = 0;
  for (int j = 0; j < n_qubits; j++) {
    int p = site_code(ax, az, j), q = site_code(bx, bz, j);
    phase += MUL_K[p][q];
    set_site(cx, cz, j, code_of_name(MUL_R[p][q]));
  }
  *k = phase % 4;
}

/* i^k as a complex number */
static void ipow(int k, double *re, double *im) {
  static const double R[4] = {1.0, 0.0, -1.0, 0.0};
  static const double I[4] = {0.0, 1.0, 0.0, -1.0};
  *re = R[((k % 4) + 4) % 4];
  *im = I[((k % 4) + 4) % 4];
}

static void cmul(double ar, double ai, double br, double bi, double *cr, double *ci) {
  double p1 = ar * br, p2 = ai * bi, p3 = ar * bi, p4 = ai * br;
  *cr = p1 - p2;
  *ci = p3 + p4;
}

static void cmul32(float ar, float ai, float br, float bi, float *cr, float *ci) {
  float p1 = ar * br, p2 = ai * bi, p3 = ar * bi, p4 = ai * br;
  *cr = p1 - p2;
  *ci = p3 + p4;
}

/* ------------------------------------------------------------------------ */
/* Key order: x word 1, x word 0, z word 1, z word 0, unsigned.              */
/* ------------------------------------------------------------------------ */
static int key_cmp(const uint64_t ax[2], const uint64_t az[2], const uint64_t bx[2],
                   const uint64_t bz[2]) {
  if (ax[1] != bx[1]) return ax[1] < bx[1] ? -1 : 1;
  if (ax[0] != bx[0]) return ax[0] < bx[0] ? -1 : 1;
  if (az[1] != bz[1]) return az[1] < bz[1] ? -1 : 1;
  if (az[0] != bz[0]) return az[0] < bz[0] ? -1 : 1;
  return 0;
}

typedef struct {
  uint64_t x[2], z[2];
  int64_t idx; /* summation order within one key */
  double re, im;
} rec_t;

static int rec_cmp(const void *pa, const void *pb) {
  const rec_t *a = (const rec_t *)pa, *b = (const rec_t *)pb;
  int c = key_cmp(a->x, a->z, b->x, b->z);
  if (c) return c;
  return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

typedef struct {
  rec_t *r;
  int64_t n, cap;
} recbuf;

static int rb_push(recbuf *b, const rec_t *r) {
  if (b->n == b->cap) {
    int64_t nc = b->cap ? 2 * b->cap : 1024;
    rec_t *p = (rec_t *)realloc(b->r, (size_t)nc * sizeof(rec_t));
    if (!p) return OR_ENOMEM;
    b->r = p;
    b->cap = nc;
  }
  b->r[b->n++] = *r;
  return OR_OK;
}

static int op_alloc(or_op *o, int n_qubits, int64_t n) {
  o->n_qubits = n_qubits;
  o->n = n;
  size_t m = (size_t)(n > 0 ? n : 1);
  o->x = (uint64_t *)calloc(2 * m, sizeof(uint64_t));
  o->z = (uint64_t *)calloc(2 * m, sizeof(uint64_t));
  o->re = (double *)calloc(m, sizeof(double));
  o->im = (double *)calloc(m, sizeof(double));
  if (!o->x || !o->z || !o->re || !o->im) return OR_ENOMEM;
  return OR_OK;
}

void or_free(or_op *op) {
  if (!op) return;
  free(op->x);
  free(op->z);
  free(op->re);
  free(op->im);
  op->x = op->z = NULL;
  op->re = op->im = NULL;
  op->n = 0;
}

static int is_zero(double re, double im) { return re == 0.0 && im == 0.0; }

/* Sort records by (key, idx) and emit one string per key, its coefficient the
 * left-to-right sum of the run; exact zeros dropped. */
static int fold_records(recbuf *b, int n_qubits, or_op *out) {
  qsort(b->r, (size_t)b->n, sizeof(rec_t), rec_cmp);
  int64_t nk = 0;
  for (int64_t i = 0; i < b->n; i++)
    if (i == 0 || key_cmp(b->r[i].x, b->r[i].z, b->r[i - 1].x, b->r[i - 1].z)) nk++;
  if (op_alloc(out, n_qubits, nk)) return OR_ENOMEM;
  int64_t m = 0;
  for (int64_t i = 0; i < b->n;) {
    int64_t j = i;
    double sr = b->r[i].re, si = b->r[i].im;
    for (j = i + 1; j < b->n && !key_cmp(b->r[j].x, b->r[j].z, b->r[i].x, b->r[i].z); j++) {
      sr = sr + b->r[j].re;
      si = si + b->r[j].im;
    }
    if (!is_zero(sr, si)) {
      memcpy(&out->x[2 * m], b->r[i].x, sizeof(b->r[i].x));
      memcpy(&out->z[2 * m], b->r[i].z, sizeof(b->r[i].z));
      out->re[m] = sr;
      out->im[m] = si;
      m++;
    }
    i = j;
  }
  out->n = m;
  return OR_OK;
}

static void get_key(const or_op *o, int64_t k, uint64_t x[2], uint64_t z[2]) {
  x[0] = o->x[2 * k];
  x[1] = o->x[2 * k + 1];
  z[0] = o->z[2 * k];
  z[1] = o->z[2 * k + 1];
}

int or_canonicalize(const or_op *in, or_op *out) {
  recbuf b = {0};
  for (int64_t k = 0; k < in->n; k++) {
    rec_t r;
    get_key(in, k, r.x, r.z);
    r.idx = k;
    r.re = in->re[k];
    r.im = in->im[k];
    if (rb_push(&b, &r)) return OR_ENOMEM;
  }
  int rc = fold_records(&b, in->n_qubits, out);
  free(b.r);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Commutator [H, O] (Alg. 1 with the commutator phase) and plain product.   */
/* ------------------------------------------------------------------------ */

/* FP32 mode with compensated sums: each contribution is the complex product
 * of the FP64 H coefficient and the stored FP32 coefficient, formed in FP64
 * and rounded once to FP32 per component, times the exact phase factor; each
 * key's contributions are summed in ascending H index with Kahan's
 * compensated summation, per component; the key's value is
 * (double)s - (double)comp. */
typedef struct {
  uint64_t x[2], z[2];
  int64_t idx;
  float re, im;
} rec32_t;

static int rec32_cmp(const void *pa, const void *pb) {
  const rec32_t *a = (const rec32_t *)pa, *b = (const rec32_t *)pb;
  int c = key_cmp(a->x, a->z, b->x, b->z);
  if (c) return c;
  return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

static void kahan_add(float *s, float *comp, float t) {
  float y = t - *comp;
  float u = *s + y;
  *comp = (u - *s) - y;
  *s = u;
}

int or_commutator(const or_op *H, const or_op *O, int prec, or_op *out) {
  int N = O->n_qubits;
  if (H->n_qubits != N || N < 1 || N > 128) return OR_EINVAL;
  if (prec == OR_F64) {
    recbuf b = {0};
    for (int64_t a = 0; a < H->n; a++) {
      uint64_t ax[2], az[2];
      get_key(H, a, ax, az);
      for (int64_t j = 0; j < O->n; j++) {
        uint64_t bx[2], bz[2], cx[2], cz[2], dx[2], dz[2];
        get_key(O, j, bx, bz);
        int kab, kba;
        or_string_product(N, ax, az, bx, bz, cx, cz, &kab);
        or_string_product(N, bx, bz, ax, az, dx, dz, &kba);
        if (kab == kba) continue; /* the strings commute */
        double pr, pi, qr, qi, dr, di;
        ipow(kab, &pr, &pi);
        ipow(kba, &qr, &qi);
        dr = pr - qr;
        di = pi - qi;
        double hr, hi;
        cmul(H->re[a], H->im[a], O->re[j], O->im[j], &hr, &hi);
        rec_t r;
        memcpy(r.x, cx, sizeof(cx));
        memcpy(r.z, cz, sizeof(cz));
        r.idx = a;
        cmul(dr, di, hr, hi, &r.re, &r.im);
        if (rb_push(&b, &r)) return OR_ENOMEM;
      }
    }
    int rc = fold_records(&b, N, out);
    free(b.r);
    return rc;
  }
  if (prec != OR_F32K) return OR_EINVAL;
  /* FP32 products, Kahan-compensated sums */
  rec32_t *rs = NULL;
  int64_t n = 0, cap = 0;
  for (int64_t a = 0; a < H->n; a++) {
    uint64_t ax[2], az[2];
    get_key(H, a, ax, az);
    for (int64_t j = 0; j < O->n; j++) {
      uint64_t bx[2], bz[2], cx[2], cz[2], dx[2], dz[2];
      get_key(O, j, bx, bz);
      int kab, kba;
      or_string_product(N, ax, az, bx, bz, cx, cz, &kab);
      or_string_product(N, bx, bz, ax, az, dx, dz, &kba);
      if (kab == kba) continue;
      double pr, pi, qr, qi;
      ipow(kab, &pr, &pi);
      ipow(kba, &qr, &qi);
      float dr = (float)(pr - qr), di = (float)(pi - qi);
      double er, ei;
      cmul(H->re[a], H->im[a], (double)(float)O->re[j], (double)(float)O->im[j], &er, &ei);
      const float tr = (float)er, ti = (float)ei;
      if (n == cap) {
        cap = cap ? 2 * cap : 1024;
        rec32_t *p = (rec32_t *)realloc(rs, (size_t)cap * sizeof(rec32_t));
        if (!p) return OR_ENOMEM;
        rs = p;
      }
      memcpy(rs[n].x, cx, sizeof(cx));
      memcpy(rs[n].z, cz, sizeof(cz));
      rs[n].idx = a;
      cmul32(dr, di, tr, ti, &rs[n].re, &rs[n].im);
      n++;
    }
  }
  qsort(rs, (size_t)n, sizeof(rec32_t), rec32_cmp);
  int64_t nk = 0;
  for (int64_t i = 0; i < n; i++)
    if (i == 0 || key_cmp(rs[i].x, rs[i].z, rs[i - 1].x, rs[i - 1].z)) nk++;
  if (op_alloc(out, N, nk)) return OR_ENOMEM;
  int64_t m = 0;
  for (int64_t i = 0; i < n;) {
    float sr = 0.0f, cr = 0.0f, si = 0.0f, ci = 0.0f;
    int64_t j = i;
    for (; j < n && !key_cmp(rs[j].x, rs[j].z, rs[i].x, rs[i].z); j++) {
      kahan_add(&sr, &cr, rs[j].re);
      kahan_add(&si, &ci, rs[j].im);
    }
    double vr = (double)sr - (double)cr, vi = (double)si - (double)ci;
    if (!is_zero(vr, vi)) {
      memcpy(&out->x[2 * m], rs[i].x, 2 * sizeof(uint64_t));
      memcpy(&out->z[2 * m], rs[i].z, 2 * sizeof(uint64_t));
      out->re[m] = vr;
      out->im[m] = vi;
      m++;
    }
    i = j;
  }
  out->n = m;
  free(rs);
  return OR_OK;
}

int or_product(const or_op *A, const or_op *B, or_op *out) {
  int N = A->n_qubits;
  if (B->n_qubits != N || N < 1 || N > 128) return OR_EINVAL;
  recbuf b = {0};
  for (int64_t a = 0; a < A->n; a++) {
    uint64_t ax[2], az[2];
    get_key(A, a, ax, az);
    for (int64_t j = 0; j < B->n; j++) {
      uint64_t bx[2], bz[2], cx[2], cz[2];
      get_key(B, j, bx, bz);
      int k;
      or_string_product(N, ax, az, bx, bz, cx, cz, &k);
      double pr, pi, hr, hi;
      ipow(k, &pr, &pi);
      cmul(A->re[a], A->im[a], B->re[j], B->im[j], &hr, &hi);
      rec_t r;
      memcpy(r.x, cx, sizeof(cx));
      memcpy(r.z, cz, sizeof(cz));
      r.idx = a;
      cmul(pr, pi, hr, hi, &r.re, &r.im);
      if (rb_push(&b, &r)) return OR_ENOMEM;
    }
  }
  int rc = fold_records(&b, N, out);
  free(b.r);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Translation-symmetric operators on a periodic chain of N sites (Alg. 2):  */
/* the operator sum_k T_k(A0) is stored as A0, one representative string per */
/* translation orbit.  T_k moves site j to site (j + k) mod N.  The          */
/* representative (Shiftleft) is the rotation whose occupied-site pattern,   */
/* read as an N-bit number with site j as bit j, is smallest; ties by the    */
/* x pattern, then the z pattern, read the same way.                         */
/* ------------------------------------------------------------------------ */
static void ts_translate(int N, const uint64_t x[2], const uint64_t z[2], int k, uint64_t ox[2],
                         uint64_t oz[2]) {
  ox[0] = ox[1] = oz[0] = oz[1] = 0;
  for (int j = 0; j < N; j++) set_site(ox, oz, (j + k) % N, site_code(x, z, j));
}

void or_ts_translate(int N, const uint64_t x[2], const uint64_t z[2], int k, uint64_t ox[2],
                     uint64_t oz[2]) {
  ts_translate(N, x, z, k, ox, oz);
}

/* 2-word numbers, most significant word first */
static int num_cmp(const uint64_t a[2], const uint64_t b[2]) {
  if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
  if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
  return 0;
}

/* Returns the rotation r (the translation by N - r, moving site r to site 0)
 * that gives the representative, the smallest r when several do. */
int or_ts_canonical(int N, const uint64_t x[2], const uint64_t z[2], uint64_t cx[2],
                    uint64_t cz[2]) {
  uint64_t bx[2] = {x[0], x[1]}, bz[2] = {z[0], z[1]};
  uint64_t bm[2] = {x[0] | z[0], x[1] | z[1]};
  int best = 0;
  for (int r = 1; r < N; r++) {
    uint64_t tx[2], tz[2];
    ts_translate(N, x, z, N - r, tx, tz);
    uint64_t tm[2] = {tx[0] | tz[0], tx[1] | tz[1]};
    int c = num_cmp(tm, bm);
    if (c == 0) c = num_cmp(tx, bx);
    if (c == 0) c = num_cmp(tz, bz);
    if (c < 0) {
      best = r;
      memcpy(bx, tx, sizeof(bx));
      memcpy(bz, tz, sizeof(bz));
      memcpy(bm, tm, sizeof(bm));
    }
  }
  memcpy(cx, bx, sizeof(bx));
  memcpy(cz, bz, sizeof(bz));
  return best;
}

/* number of k in [0, N) with T_k(s) = s */
static int ts_stabilizer(int N, const uint64_t x[2], const uint64_t z[2]) {
  int s = 0;
  for (int k = 0; k < N; k++) {
    uint64_t tx[2], tz[2];
    ts_translate(N, x, z, k, tx, tz);
    if (!key_cmp(tx, tz, x, z)) s++;
  }
  return s;
}

/* [H, O] for H = sum_k T_k(H0) and O = sum_k T_k(O0): H0 expanded to the list
 * T_0(h_0), T_1(h_0), ..., T_{N-1}(h_0), T_0(h_1), ..., every anticommuting
 * pair with an O0 string gives 2 i^e h c on the representative of its
 * product.  Summation order per representative: ascending list entry, then
 * ascending rotation r of the product (one O0 string per entry and r). */
int or_commutator_ts(const or_op *H0, const or_op *O, or_op *out) {
  int N = O->n_qubits;
  if (H0->n_qubits != N || N < 1 || N > 128) return OR_EINVAL;
  recbuf b = {0};
  for (int64_t a = 0; a < H0->n; a++) {
    uint64_t hx[2], hz[2];
    get_key(H0, a, hx, hz);
    for (int k = 0; k < N; k++) {
      uint64_t ax[2], az[2];
      ts_translate(N, hx, hz, k, ax, az);
      for (int64_t j = 0; j < O->n; j++) {
        uint64_t bx[2], bz[2], cx[2], cz[2], dx[2], dz[2];
        get_key(O, j, bx, bz);
        int kab, kba;
        or_string_product(N, ax, az, bx, bz, cx, cz, &kab);
        or_string_product(N, bx, bz, ax, az, dx, dz, &kba);
        if (kab == kba) continue;
        double pr, pi, qr, qi, dr, di, hr, hi;
        ipow(kab, &pr, &pi);
        ipow(kba, &qr, &qi);
        dr = pr - qr;
        di = pi - qi;
        cmul(H0->re[a], H0->im[a], O->re[j], O->im[j], &hr, &hi);
        rec_t r;
        const int rot = or_ts_canonical(N, cx, cz, r.x, r.z);
        r.idx = (a * N + k) * 256 + rot;
        cmul(dr, di, hr, hi, &r.re, &r.im);
        if (rb_push(&b, &r)) return OR_ENOMEM;
      }
    }
  }
  int rc = fold_records(&b, N, out);
  free(b.r);
  return rc;
}

/* ||sum_k T_k(A0)||^2 / N = sum over representatives of stab(s) |c_s|^2,
 * exactly accumulated and rounded once (A0: one string per orbit). */
double or_norm2_ts(const or_op *A) {
  int *st = (int *)malloc((size_t)(A->n > 0 ? A->n : 1) * sizeof(int));
  if (!st) return -1.0;
  int64_t m = 0;
  for (int64_t k = 0; k < A->n; k++) {
    uint64_t x[2], z[2];
    get_key(A, k, x, z);
    st[k] = ts_stabilizer(A->n_qubits, x, z);
    m += st[k];
  }
  double *v = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
  if (!v) {
    free(st);
    return -1.0;
  }
  int64_t t = 0;
  for (int64_t k = 0; k < A->n; k++) {
    const double w = A->re[k] * A->re[k] + A->im[k] * A->im[k];
    for (int r = 0; r < st[k]; r++) v[t++] = w;
  }
  double r = or_exact_sum(v, m);
  free(v);
  free(st);
  return r;
}

/* ------------------------------------------------------------------------ */
/* alpha A + beta B: fl(fl(alpha a) + fl(beta b)); a missing side adds nothing */
/* ------------------------------------------------------------------------ */
int or_add(const or_op *A, double ar, double ai, const or_op *B, double br, double bi,
           or_op *out) {
  if (A->n_qubits != B->n_qubits) return OR_EINVAL;
  recbuf b = {0};
  for (int64_t k = 0; k < A->n; k++) {
    rec_t r;
    get_key(A, k, r.x, r.z);
    r.idx = 0;
    cmul(ar, ai, A->re[k], A->im[k], &r.re, &r.im);
    if (rb_push(&b, &r)) return OR_ENOMEM;
  }
  for (int64_t k = 0; k < B->n; k++) {
    rec_t r;
    get_key(B, k, r.x, r.z);
    r.idx = 1;
    cmul(br, bi, B->re[k], B->im[k], &r.re, &r.im);
    if (rb_push(&b, &r)) return OR_ENOMEM;
  }
  int rc = fold_records(&b, A->n_qubits, out);
  free(b.r);
  return rc;
}

int or_divide(const or_op *in, double b, or_op *out) {
  if (op_alloc(out, in->n_qubits, in->n)) return OR_ENOMEM;
  int64_t m = 0;
  for (int64_t k = 0; k < in->n; k++) {
    double re = in->re[k] / b, im = in->im[k] / b;
    if (is_zero(re, im)) continue;
    memcpy(&out->x[2 * m], &in->x[2 * k], 2 * sizeof(uint64_t));
    memcpy(&out->z[2 * m], &in->z[2 * k], 2 * sizeof(uint64_t));
    out->re[m] = re;
    out->im[m] = im;
    m++;
  }
  out->n = m;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Truncation                                                                */
/* ------------------------------------------------------------------------ */
static int string_length(const uint64_t x[2], const uint64_t z[2], int n_qubits) {
  int len = 0;
  for (int j = 0; j < n_qubits; j++)
    if (site_code(x, z, j) != 0) len++;
  return len;
}

/* Depolarizing noise (Heisenberg time evolution section): the string of
 * length w is transmitted with rate exp(-lambda w), lambda = eps dt per step.
 * Each coefficient is multiplied by that factor; exact zeros are dropped. */
int or_add_noise(const or_op *in, double lambda, or_op *out) {
  if (op_alloc(out, in->n_qubits, in->n)) return OR_ENOMEM;
  int64_t m = 0;
  for (int64_t k = 0; k < in->n; k++) {
    uint64_t x[2], z[2];
    get_key(in, k, x, z);
    const double f = exp(-lambda * (double)string_length(x, z, in->n_qubits));
    double re = in->re[k] * f, im = in->im[k] * f;
    if (is_zero(re, im)) continue;
    memcpy(&out->x[2 * m], x, 2 * sizeof(uint64_t));
    memcpy(&out->z[2 * m], z, 2 * sizeof(uint64_t));
    out->re[m] = re;
    out->im[m] = im;
    m++;
  }
  out->n = m;
  return OR_OK;
}

static int in_keep(const or_op *keep, const uint64_t x[2], const uint64_t z[2]) {
  if (!keep) return 0;
  for (int64_t k = 0; k < keep->n; k++) {
    uint64_t kx[2], kz[2];
    get_key(keep, k, kx, kz);
    if (!key_cmp(kx, kz, x, z)) return 1;
  }
  return 0;
}

typedef struct {
  double m2;
  uint64_t x[2], z[2];
  int64_t src;
} cand_t;

/* larger weight first; equal weights: smaller key first */
static int cand_cmp(const void *pa, const void *pb) {
  const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
  if (a->m2 != b->m2) return a->m2 > b->m2 ? -1 : 1;
  return key_cmp(a->x, a->z, b->x, b->z);
}

static int out_key_cmp(const void *pa, const void *pb) {
  const rec_t *a = (const rec_t *)pa, *b = (const rec_t *)pb;
  return key_cmp(a->x, a->z, b->x, b->z);
}

int or_truncate(const or_op *in, const or_trunc *t, or_op *out) {
  int N = in->n_qubits;
  double eps2 = t->coef_eps * t->coef_eps;
  rec_t *kept = (rec_t *)malloc(sizeof(rec_t) * (size_t)(in->n + 1));
  cand_t *rest = (cand_t *)malloc(sizeof(cand_t) * (size_t)(in->n + 1));
  if (!kept || !rest) return OR_ENOMEM;
  int64_t nf = 0, nr = 0;
  for (int64_t k = 0; k < in->n; k++) {
    uint64_t x[2], z[2];
    get_key(in, k, x, z);
    double re = in->re[k], im = in->im[k];
    if (is_zero(re, im)) continue;
    if (t->max_len > 0 && string_length(x, z, N) > t->max_len) continue;
    double m2 = re * re + im * im; /* two rounded squares, one rounded sum */
    if (t->coef_eps > 0.0 && !(m2 >= eps2)) continue;
    if (in_keep(t->keep, x, z)) {
      memcpy(kept[nf].x, x, sizeof(x));
      memcpy(kept[nf].z, z, sizeof(z));
      kept[nf].re = re;
      kept[nf].im = im;
      nf++;
    } else {
      rest[nr].m2 = m2;
      memcpy(rest[nr].x, x, sizeof(x));
      memcpy(rest[nr].z, z, sizeof(z));
      rest[nr].src = k;
      nr++;
    }
  }
  int64_t take = nr;
  if (t->max_strings > 0) {
    int64_t budget = t->max_strings - nf;
    if (budget < 0) budget = 0;
    if (budget < nr) {
      qsort(rest, (size_t)nr, sizeof(cand_t), cand_cmp);
      take = budget;
    }
  }
  for (int64_t k = 0; k < take; k++) {
    int64_t s = rest[k].src;
    memcpy(kept[nf].x, rest[k].x, sizeof(rest[k].x));
    memcpy(kept[nf].z, rest[k].z, sizeof(rest[k].z));
    kept[nf].re = in->re[s];
    kept[nf].im = in->im[s];
    nf++;
  }
  qsort(kept, (size_t)nf, sizeof(rec_t), out_key_cmp);
  if (op_alloc(out, N, nf)) return OR_ENOMEM;
  for (int64_t k = 0; k < nf; k++) {
    memcpy(&out->x[2 * k], kept[k].x, 2 * sizeof(uint64_t));
    memcpy(&out->z[2 * k], kept[k].z, 2 * sizeof(uint64_t));
    out->re[k] = kept[k].re;
    out->im[k] = kept[k].im;
  }
  free(kept);
  free(rest);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Exact summation: a two's-complement fixed-point integer in units of       */
/* 2^-1074 (the smallest subnormal), wide enough for any sum of < 2^400      */
/* finite doubles; rounded once to nearest-even at the end.                  */
/* ------------------------------------------------------------------------ */
#define XLIMBS 40
typedef struct {
  uint64_t w[XLIMBS];
} xacc;

static void xacc_add(xacc *a, double d) {
  if (d == 0.0 || d != d) return;
  int neg = d < 0.0;
  int e;
  double f = frexp(fabs(d), &e);        /* |d| = f 2^e, 0.5 <= f < 1 */
  uint64_t m = (uint64_t)ldexp(f, 53);  /* exact, 2^52 <= m < 2^53   */
  int s = e - 53 + 1074;                /* |d| = m 2^(s-1074)         */
  if (s < 0) {                          /* subnormal: shifted-out bits are zero */
    m >>= -s;
    s = 0;
  }
  int limb = s / 64, off = s % 64;
  uint64_t part[2];
  part[0] = m << off;
  part[1] = off ? (m >> (64 - off)) : 0;
  if (!neg) {
    uint64_t carry = 0;
    for (int i = limb; i < XLIMBS; i++) {
      uint64_t add = (i - limb < 2) ? part[i - limb] : 0;
      uint64_t s1 = a->w[i] + add;
      uint64_t c1 = s1 < add;
      uint64_t s2 = s1 + carry;
      uint64_t c2 = s2 < carry;
      a->w[i] = s2;
      carry = c1 | c2;
      if (i - limb >= 1 && !carry) break;
    }
  } else {
    uint64_t borrow = 0;
    for (int i = limb; i < XLIMBS; i++) {
      uint64_t sub = (i - limb < 2) ? part[i - limb] : 0;
      uint64_t v = a->w[i];
      uint64_t d1 = v - sub;
      uint64_t b1 = v < sub;
      uint64_t d2 = d1 - borrow;
      uint64_t b2 = d1 < borrow;
      a->w[i] = d2;
      borrow = b1 | b2;
      if (i - limb >= 1 && !borrow) break;
    }
  }
}

static double xacc_round(const xacc *a) {
  uint64_t w[XLIMBS];
  memcpy(w, a->w, sizeof(w));
  int neg = (int)(w[XLIMBS - 1] >> 63);
  if (neg) { /* two's complement negate */
    uint64_t carry = 1;
    for (int i = 0; i < XLIMBS; i++) {
      uint64_t v = ~w[i] + carry;
      carry = (carry && v == 0) ? 1 : 0;
      w[i] = v;
    }
  }
  int top = -1;
  for (int i = XLIMBS - 1; i >= 0 && top < 0; i--)
    if (w[i]) top = i * 64 + 63 - __builtin_clzll(w[i]);
  if (top < 0) return 0.0;
#define BIT(p) ((int)((w[(p) / 64] >> ((p) % 64)) & 1u))
  uint64_t mant = 0;
  int lo = top - 52; /* lowest bit kept */
  if (lo < 0) lo = 0;
  for (int p = top; p >= lo; p--) mant = (mant << 1) | (uint64_t)BIT(p);
  if (lo > 0) {
    int guard = BIT(lo - 1);
    int sticky = 0;
    for (int p = lo - 2; p >= 0 && !sticky; p--) sticky = BIT(p);
    if (guard && (sticky || (mant & 1u))) mant++;
  }
#undef BIT
  double r = ldexp((double)mant, lo - 1074);
  return neg ? -r : r;
}

double or_exact_sum(const double *v, int64_t n) {
  xacc a;
  memset(&a, 0, sizeof(a));
  for (int64_t i = 0; i < n; i++) xacc_add(&a, v[i]);
  return xacc_round(&a);
}

/* ||A||^2 = sum_k fl(fl(re^2) + fl(im^2)), summed exactly, rounded once */
double or_norm2(const or_op *A) {
  xacc a;
  memset(&a, 0, sizeof(a));
  for (int64_t k = 0; k < A->n; k++) {
    double m2 = A->re[k] * A->re[k] + A->im[k] * A->im[k];
    xacc_add(&a, m2);
  }
  return xacc_round(&a);
}

/* <A,B> = sum over common keys of conj(a) b; every rounded elementary product
 * fl(ar br), fl(ai bi), fl(ar bi), -fl(ai br) is summed exactly, rounded once. */
void or_inner(const or_op *A, const or_op *B, double *re, double *im) {
  xacc sr, si;
  memset(&sr, 0, sizeof(sr));
  memset(&si, 0, sizeof(si));
  for (int64_t i = 0; i < A->n; i++) {
    uint64_t ax[2], az[2];
    get_key(A, i, ax, az);
    for (int64_t j = 0; j < B->n; j++) {
      uint64_t bx[2], bz[2];
      get_key(B, j, bx, bz);
      if (key_cmp(ax, az, bx, bz)) continue;
      xacc_add(&sr, A->re[i] * B->re[j]);
      xacc_add(&sr, A->im[i] * B->im[j]);
      xacc_add(&si, A->re[i] * B->im[j]);
      xacc_add(&si, -(A->im[i] * B->re[j]));
    }
  }
  *re = xacc_round(&sr);
  *im = xacc_round(&si);
}

/* ------------------------------------------------------------------------ */
/* Lanczos step (Krylov section; the printed lanczos listing):               */
/*   O'_n = [H, O_{n-1}] - b_{n-1} O_{n-2}   (no second term at n = 1)      */
/*   b_n  = ||O'_n|| = sqrt(sum |c|^2)       (norm of the untruncated O'_n) */
/*   O_n  = trunc(O'_n / b_n)                                                */
/* Breakdown when b_n <= 1e-13 max(1, b_{n-1}).                              */
/* prec = OR_F32K: commutator in FP32 with Kahan sums (values then FP64),    */
/* recombination, norm, division and truncation decisions in FP64, the kept */
/* values rounded to FP32.                                                   */
/* ------------------------------------------------------------------------ */
static void round_to_f32(or_op *o) {
  int64_t m = 0;
  for (int64_t k = 0; k < o->n; k++) {
    double re = (double)(float)o->re[k], im = (double)(float)o->im[k];
    if (is_zero(re, im)) continue;
    memmove(&o->x[2 * m], &o->x[2 * k], 2 * sizeof(uint64_t));
    memmove(&o->z[2 * m], &o->z[2 * k], 2 * sizeof(uint64_t));
    o->re[m] = re;
    o->im[m] = im;
    m++;
  }
  o->n = m;
}

static void drop_f32_zeros(or_op *o) {
  int64_t m = 0;
  for (int64_t k = 0; k < o->n; k++) {
    if (is_zero((double)(float)o->re[k], (double)(float)o->im[k])) continue;
    memmove(&o->x[2 * m], &o->x[2 * k], 2 * sizeof(uint64_t));
    memmove(&o->z[2 * m], &o->z[2 * k], 2 * sizeof(uint64_t));
    o->re[m] = o->re[k];
    o->im[m] = o->im[k];
    m++;
  }
  o->n = m;
}

/* ts != 0: translation-symmetric operators of the periodic chain (Alg. 2):  */
/* H holds H0, the operators hold orbit representatives, the commutator is   */
/* or_commutator_ts and the norm the stabilizer-weighted or_norm2_ts (FP64). */
/* reorth != 0: local re-orthogonalisation (not in the paper; its recursion */
/* is the three-term one): O'_n is replaced by                               */
/*   O'_n - a_1 O_{n-1} - a_2 O_{n-2},  a_k = <O_k, O'_n> / <O_k, O_k>,      */
/* both a_k from the same O'_n (Gram-Schmidt against the two previous        */
/* vectors), inner products and norms exact sums rounded once, the           */
/* combination by two sums (O'_n + (-a_1) O_{n-1}) + (-a_2) O_{n-2}.         */
static int project_out(or_op *A, const or_op *const V[2]) {
  double ar[2] = {0.0, 0.0}, ai[2] = {0.0, 0.0};
  for (int k = 0; k < 2; k++) {
    if (!V[k] || V[k]->n == 0) continue;
    double n2 = or_norm2(V[k]), re, im;
    or_inner(V[k], A, &re, &im);
    if (n2 > 0.0) {
      ar[k] = re / n2;
      ai[k] = im / n2;
    }
  }
  for (int k = 0; k < 2; k++) {
    if (!V[k] || V[k]->n == 0) continue;
    or_op B = {0};
    int rc = or_add(A, 1.0, 0.0, V[k], -ar[k], -ai[k], &B);
    if (rc) return rc;
    or_free(A);
    *A = B;
  }
  return OR_OK;
}

static int lanczos_step(int ts, const or_op *H, const or_op *O_prev, const or_op *O_cur,
                        double b_prev, const or_trunc *t, int prec, int reorth, or_op *O_next,
                        double *b_out) {
  or_op C = {0}, A = {0}, D = {0};
  int rc = ts ? or_commutator_ts(H, O_cur, &C) : or_commutator(H, O_cur, prec, &C);
  if (rc) return rc;
  if (O_prev && O_prev->n > 0) {
    rc = or_add(&C, 1.0, 0.0, O_prev, -b_prev, 0.0, &A);
    or_free(&C);
    if (rc) return rc;
  } else {
    A = C;
  }
  if (reorth) {
    const or_op *V[2] = {O_cur, O_prev};
    rc = project_out(&A, V);
    if (rc) {
      or_free(&A);
      return rc;
    }
  }
  double b = sqrt(ts ? or_norm2_ts(&A) : or_norm2(&A));
  *b_out = b;
  double floor_b = 1e-13 * (b_prev > 1.0 ? b_prev : 1.0);
  if (!(b > floor_b)) {
    or_free(&A);
    op_alloc(O_next, H->n_qubits, 0);
    return OR_BREAKDOWN;
  }
  rc = or_divide(&A, b, &D);
  or_free(&A);
  if (rc) return rc;
  /* FP32 mode: strings whose FP32 value would be an exact zero are dropped;
   * the cutoff and top-M are decided on the FP64 quotient; the kept values
   * are then rounded to FP32 */
  if (prec == OR_F32K) drop_f32_zeros(&D);
  rc = or_truncate(&D, t, O_next);
  or_free(&D);
  if (rc == OR_OK && prec == OR_F32K) round_to_f32(O_next);
  return rc;
}

int or_lanczos_step(const or_op *H, const or_op *O_prev, const or_op *O_cur, double b_prev,
                    const or_trunc *t, int prec, or_op *O_next, double *b_out) {
  return lanczos_step(0, H, O_prev, O_cur, b_prev, t, prec, 0, O_next, b_out);
}

int or_lanczos_step_reorth(const or_op *H, const or_op *O_prev, const or_op *O_cur,
                           double b_prev, const or_trunc *t, int prec, or_op *O_next,
                           double *b_out) {
  return lanczos_step(0, H, O_prev, O_cur, b_prev, t, prec, 1, O_next, b_out);
}

int or_lanczos_step_ts(const or_op *H0, const or_op *O_prev, const or_op *O_cur, double b_prev,
                       const or_trunc *t, or_op *O_next, double *b_out) {
  return lanczos_step(1, H0, O_prev, O_cur, b_prev, t, OR_F64, 0, O_next, b_out);
}

/* ------------------------------------------------------------------------ */
/* Classical 4-stage Runge-Kutta step of dO/dt = i[H, O] (Heisenberg         */
/* evolution section), truncating every stage input and the result:          */
/*   k1 = i[H,O]          S2 = trunc(O + (dt/2) k1)                          */
/*   k2 = i[H,S2]         S3 = trunc(O + (dt/2) k2)                          */
/*   k3 = i[H,S3]         S4 = trunc(O + dt k3)                              */
/*   k4 = i[H,S4]         O' = trunc(((((O + c1 k1) + c2 k2) + c2 k3) + c1 k4)) */
/* with c1 = fl(dt/6), c2 = fl(dt/3); multiplying by i is exact.             */
/* ------------------------------------------------------------------------ */
static int times_i_commutator(const or_op *H, const or_op *S, or_op *k) {
  int rc = or_commutator(H, S, OR_F64, k);
  if (rc) return rc;
  for (int64_t j = 0; j < k->n; j++) {
    double re = k->re[j], im = k->im[j];
    k->re[j] = -im;
    k->im[j] = re;
  }
  return OR_OK;
}

int or_rk4_step(const or_op *H, const or_op *O, double dt, const or_trunc *t, or_op *out) {
  double h2 = dt / 2.0, c1 = dt / 6.0, c2 = dt / 3.0;
  or_op k1 = {0}, k2 = {0}, k3 = {0}, k4 = {0}, S = {0}, T = {0}, A = {0}, B = {0};
  int rc;
  if ((rc = times_i_commutator(H, O, &k1))) return rc;
  if ((rc = or_add(O, 1.0, 0.0, &k1, h2, 0.0, &T))) return rc;
  if ((rc = or_truncate(&T, t, &S))) return rc;
  or_free(&T);
  if ((rc = times_i_commutator(H, &S, &k2))) return rc;
  or_free(&S);
  if ((rc = or_add(O, 1.0, 0.0, &k2, h2, 0.0, &T))) return rc;
  if ((rc = or_truncate(&T, t, &S))) return rc;
  or_free(&T);
  if ((rc = times_i_commutator(H, &S, &k3))) return rc;
  or_free(&S);
  if ((rc = or_add(O, 1.0, 0.0, &k3, dt, 0.0, &T))) return rc;
  if ((rc = or_truncate(&T, t, &S))) return rc;
  or_free(&T);
  if ((rc = times_i_commutator(H, &S, &k4))) return rc;
  or_free(&S);
  if ((rc = or_add(O, 1.0, 0.0, &k1, c1, 0.0, &A))) return rc;
  if ((rc = or_add(&A, 1.0, 0.0, &k2, c2, 0.0, &B))) return rc;
  or_free(&A);
  if ((rc = or_add(&B, 1.0, 0.0, &k3, c2, 0.0, &A))) return rc;
  or_free(&B);
  if ((rc = or_add(&A, 1.0, 0.0, &k4, c1, 0.0, &B))) return rc;
  or_free(&A);
  rc = or_truncate(&B, t, out);
  or_free(&B);
  or_free(&k1);
  or_free(&k2);
  or_free(&k3);
  or_free(&k4);
  return rc;
}
