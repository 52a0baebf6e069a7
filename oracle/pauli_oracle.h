/* Plain CPU oracle for the Pauli-string operator algebra.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this library; the product
 * path (the HIP library and its Python binding) never does.  It shares no
 * code with the HIP path: it multiplies strings site by site with the
 * textbook single-site Pauli table instead of the popcount formulas, keeps
 * its operators as plain arrays sorted by key, sums with qsort + sequential
 * folds, and rounds norms from an exact fixed-point accumulator.
 *
 * Operators: sum_k (re[k] + i im[k]) P(x[k], z[k]) on n_qubits <= 128 sites;
 * x and z are arrays of [n][2] words (site j, 1-based, is bit (j-1)%64 of
 * word (j-1)/64); I=(0,0) X=(1,0) Z=(0,1) Y=(1,1), every P Hermitian.
 * Outputs are malloc'ed by the oracle (free with or_free) and sorted by key:
 * x word 1, x word 0, z word 1, z word 0, each compared as unsigned.
 */
#ifndef PAULI_ORACLE_H
#define PAULI_ORACLE_H
#include <stdint.h>

typedef struct {
  int32_t n_qubits;
  int64_t n;
  uint64_t *x; /* [n][2] */
  uint64_t *z; /* [n][2] */
  double *re;  /* [n] */
  double *im;  /* [n] */
} or_op;

typedef struct {
  int32_t max_len;      /* <= 0: no length cap */
  double coef_eps;      /* drop |c| < eps; exact zeros are always dropped */
  int64_t max_strings;  /* <= 0: no top-M */
  const or_op *keep;    /* nullable; strings never removed by top-M */
} or_trunc;

enum { OR_OK = 0, OR_EINVAL = 1, OR_ENOMEM = 2, OR_BREAKDOWN = 4 };
enum { OR_F64 = 0, OR_F32K = 1 };

void or_free(or_op *op);

/* single-string product P_a P_b = i^k P_c with the site-by-site table */
void or_string_product(int n_qubits, const uint64_t ax[2], const uint64_t az[2],
                       const uint64_t bx[2], const uint64_t bz[2],
                       uint64_t cx[2], uint64_t cz[2], int *k);

/* sum duplicates in input order, drop exact zeros, sort by key */
int or_canonicalize(const or_op *in, or_op *out);
/* [H, O]; each output coefficient sums its contributions in ascending H index */
int or_commutator(const or_op *H, const or_op *O, int prec, or_op *out);
/* plain product H O (Alg. 1 with the string-product phase) */
int or_product(const or_op *A, const or_op *B, or_op *out);
/* alpha A + beta B over the union of keys */
int or_add(const or_op *A, double ar, double ai, const or_op *B, double br, double bi,
           or_op *out);
int or_truncate(const or_op *in, const or_trunc *t, or_op *out);
int or_divide(const or_op *in, double b, or_op *out);
int or_add_noise(const or_op *in, double lambda, or_op *out);
int or_ts_canonical(int N, const uint64_t x[2], const uint64_t z[2], uint64_t cx[2],
                    uint64_t cz[2]);
void or_ts_translate(int N, const uint64_t x[2], const uint64_t z[2], int k, uint64_t ox[2],
                     uint64_t oz[2]);
int or_commutator_ts(const or_op *H0, const or_op *O, or_op *out);
double or_norm2_ts(const or_op *A);
double or_norm2(const or_op *A);
void or_inner(const or_op *A, const or_op *B, double *re, double *im);
double or_exact_sum(const double *v, int64_t n);
int or_lanczos_step(const or_op *H, const or_op *O_prev, const or_op *O_cur, double b_prev,
                    const or_trunc *t, int prec, or_op *O_next, double *b_out);
/* the same step with local re-orthogonalisation against O_cur and O_prev */
int or_lanczos_step_reorth(const or_op *H, const or_op *O_prev, const or_op *O_cur,
                           double b_prev, const or_trunc *t, int prec, or_op *O_next,
                           double *b_out);
int or_lanczos_step_ts(const or_op *H0, const or_op *O_prev, const or_op *O_cur, double b_prev,
                       const or_trunc *t, or_op *O_next, double *b_out);
int or_rk4_step(const or_op *H, const or_op *O, double dt, const or_trunc *t, or_op *out);

#endif
