/* pauli.h - C ABI of the MI355X (gfx950) Pauli-string operator engine.
 *
 * An operator is a sum of Pauli strings, O = sum_k c_k P(x_k, z_k), each
 * string encoded in binary as two bit-masks (Methods, "Pauli strings": the
 * encoding of strings as pairs of integers whose product is an XOR of the
 * masks with a phase from popcounts).  Site j (1-based) is bit (j-1) % 64 of
 * word (j-1) / 64; I=(x,z)=(0,0), X=(1,0), Z=(0,1), Y=(1,1), and P(x,z) is the
 * Hermitian tensor product of those Paulis (so the paper's tau_11 = iY is
 * represented as i * Y).
 *
 * Memory and ownership
 *   - Every pointer inside pauli_op and pauli_ws is a DEVICE pointer owned by
 *     the caller.  The library never allocates or frees device memory and
 *     keeps no pointer to caller memory after a call returns.  State kept
 *     between calls: a pinned host control block (under 1 KiB) per calling thread
 *     (allocated with hipHostMalloc on the thread's first call, kept until the
 *     process ends), two events and a side stream of default priority per
 *     calling thread (created on its first call, on the device then current;
 *     the control block is copied to the host on the side stream while the
 *     call's own stream goes on), the per-thread diagnostics below and the
 *     optional kernel-timing log (pauli_profile_*).
 *   - x and z are word-major: word w of string k is x[w * capacity + k].
 *     coef holds `capacity` interleaved (re, im) pairs: double for
 *     PAULI_C128, float for PAULI_C64K.
 *   - Inputs are read-only.  An output must not alias any input.
 *   - Calls enqueue work on `stream` (a hipStream_t) and synchronise it
 *     before returning, so sizes and scalars are valid on return.
 *
 * Canonical form
 *   Every operator the library writes is canonical: unique strings, no exact
 *   zero coefficient, sorted in the library's fixed order (ascending value of
 *   a bijective mix of the key words).  Operators built elsewhere are brought
 *   to this form with pauli_canonicalize.  Inputs of pauli_commutator,
 *   pauli_add, pauli_truncate and the step functions need unique strings but
 *   may come in any order; the keep set of a pauli_trunc and the second
 *   argument of pauli_inner must be canonical.
 *
 * Summation order (determinism)
 *   Each output coefficient of a commutator sums its contributions in
 *   ascending index of the H string that produced it; a linear combination
 *   alpha A + beta B is fl(fl(alpha a) + fl(beta b)); norms are sums of
 *   fl(fl(re^2) + fl(im^2)) accumulated in double-double and rounded once.
 *   Results are bitwise reproducible run to run.
 *
 * Errors
 *   Every function returns a pauli_status.  PAULI_ECAPACITY: an output's
 *   capacity is too small; its `size` field receives the required number of
 *   strings and no output is valid.  PAULI_EWORKSPACE: the workspace is too
 *   small; ws->required receives a sufficient size in bytes (retry with at
 *   least that much; data-dependent sizes may need one more retry).
 *   PAULI_BREAKDOWN: a Lanczos step produced b_n <= 1e-13 max(1, b_{n-1}).
 *   PAULI_EHIP: a HIP runtime error (text from pauli_last_error()).
 */
#ifndef PAULI_H
#define PAULI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PAULI_OK = 0,
  PAULI_EINVAL = 1,
  PAULI_ECAPACITY = 2,
  PAULI_EWORKSPACE = 3,
  PAULI_BREAKDOWN = 4,
  PAULI_EHIP = 5,
  PAULI_EINTERNAL = 6
} pauli_status;

typedef enum {
  PAULI_C128 = 0, /* complex double coefficients */
  PAULI_C64K = 1  /* complex float coefficients; products in FP32 with
                     Kahan-compensated sums, recombination, norms and b_n in
                     FP64 (precision split of the Lanczos recursion) */
} pauli_dtype;

typedef struct pauli_op {
  int32_t n_qubits;  /* 1..128 */
  int32_t dtype;     /* pauli_dtype */
  int64_t size;      /* strings in use; written by the library on outputs */
  int64_t capacity;  /* rows allocated for x, z and coef */
  uint64_t *x;       /* device, [W][capacity], W = (n_qubits + 63) / 64 */
  uint64_t *z;       /* device, [W][capacity] */
  void *coef;        /* device, [capacity] (re, im) */
} pauli_op;

/* Truncation (Methods: keeping only the strings of largest weight; discarding
 * long strings; the cutoff of the Lanczos listing), applied in this order:
 *   1. drop strings with popcount(x | z) > max_len        (max_len <= 0: off)
 *   2. drop strings with |c| < coef_eps, compared as
 *      fl(fl(re^2)+fl(im^2)) < fl(coef_eps^2); exact zeros always dropped
 *   3. keep every surviving string of `keep`, then the
 *      max(0, max_strings - kept) largest |c| among the rest, ties broken by
 *      the smaller key (x words from high to low, then z words from high to
 *      low, unsigned)                                      (max_strings <= 0: off)
 */
typedef struct pauli_trunc {
  int32_t max_len;
  double coef_eps;
  int64_t max_strings;
  const pauli_op *keep; /* nullable; canonical; at most 65536 strings */
} pauli_trunc;

typedef struct pauli_ws {
  void *ptr;       /* device scratch, 256-byte aligned */
  size_t bytes;
  size_t required; /* written on PAULI_EWORKSPACE */
} pauli_ws;

/* out = [H, O] = sum_{a,b} h_a c_b [P_a, P_b] (Alg. 1 in commutator form with
 * the commutator phase of eq. eps_com), then truncated by t (nullable: only
 * exact zeros are dropped).  H must be PAULI_C128; O and out share a dtype. */
int pauli_commutator(const pauli_op *H, const pauli_op *O, const pauli_trunc *t,
                     pauli_op *out, pauli_ws *ws, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): pauli_commutator with its
 * scratch in a static device array of 256 MiB per GPU (held from the first
 * call on that GPU until the process ends) instead of a caller workspace.
 * Allocates no device or pinned host memory.  Inputs, output and errors as
 * pauli_commutator; a call whose scratch exceeds 256 MiB returns
 * PAULI_EWORKSPACE (pauli_last_error names the need) and writes no output.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (several host threads or streams) race and must be serialised by the
 * caller.  Synchronous at return, like pauli_commutator. */
int pauli_commutator_noalloc(const pauli_op *H, const pauli_op *O, const pauli_trunc *t,
                             pauli_op *out, void *stream);

/* out = trunc(A B) = sum_{a,b} a_a b_b P_a P_b (Alg. 1 as written: every pair,
 * the string product and phase of the single-site multiplication table),
 * summed per string in ascending index of A.  A must be PAULI_C128 with fewer
 * strings than one merge bucket holds (as H of pauli_commutator); B and out
 * share a dtype.  Pairs are not filtered, so the records number |A| |B|. */
int pauli_multiply(const pauli_op *A, const pauli_op *B, const pauli_trunc *t,
                   pauli_op *out, pauli_ws *ws, void *stream);

/* Translation-symmetric operators on a periodic chain of N = n_qubits sites
 * (Methods, Alg. 2): the operator sum_k T_k(A0), T_k moving site j to
 * (j + k) mod N, is held as A0 with one representative string per
 * translation orbit.  The representative of a string is its rotation whose
 * occupied-site pattern (x | z, site j = bit j) is the smallest N-bit number,
 * ties by x, then z (it starts on the first site).
 *
 * pauli_commutator_ts1d: representatives of trunc([sum_k T_k(H0), sum_k T_k(O)])
 * = sum over k, h, o of [T_k(h), o] with every product replaced by its
 * representative; H0 is listed over its translations as T_0(h_0), ...,
 * T_{N-1}(h_0), T_0(h_1), ... and each string's contributions are summed in
 * that order.  O must hold representatives (pauli_canonicalize_ts1d);
 * H0 any strings (PAULI_C128, N |H0| below one merge bucket's capacity).
 * pauli_canonicalize_ts1d: every string replaced by its representative,
 * duplicates summed in input order, canonical order.
 * pauli_norm2_ts1d: *out (host) = ||sum_k T_k(A)||^2 / N = sum over A's
 * representatives of stab(s)|c_s|^2 (stab: translations leaving s unchanged);
 * the b_n of a Lanczos recursion are the same under this norm.
 * pauli_lanczos_step_ts1d: pauli_lanczos_step on translation-symmetric
 * operators (the Krylov section's recursion with the commutator above and
 * this norm): O'_n = [sum_k T_k(H0), O_cur] - b_prev O_prev as
 * representatives, *b_out = sqrt(pauli_norm2_ts1d(O'_n)), O_next =
 * trunc(O'_n / b_n); the same errors and breakdown rule as
 * pauli_lanczos_step.  With O_0 of unit norm the b_n are those of the plain
 * recursion on the full periodic-chain operators. */
int pauli_commutator_ts1d(const pauli_op *H0, const pauli_op *O, const pauli_trunc *t,
                          pauli_op *out, pauli_ws *ws, void *stream);
int pauli_canonicalize_ts1d(const pauli_op *in, pauli_op *out, pauli_ws *ws, void *stream);
int pauli_norm2_ts1d(const pauli_op *A, double *out, pauli_ws *ws, void *stream);
int pauli_lanczos_step_ts1d(const pauli_op *H0, const pauli_op *O_prev, const pauli_op *O_cur,
                            double b_prev, const pauli_trunc *t, pauli_op *O_next,
                            double *b_out, pauli_ws *ws, void *stream);

/* out[0] + i out[1] (host) = Tr(A)/2^N: the coefficient of the identity string
 * (0 when A has none).  A's strings must be distinct.  With pauli_multiply it
 * gives the moments Tr(H^k)/2^N of the Conclusion's spectral outlook. */
int pauli_trace(const pauli_op *A, double out[2], pauli_ws *ws, void *stream);

/* out = trunc(alpha A + beta B) over the union of strings (the operator sum
 * used by both the Lanczos recursion and the Runge-Kutta stages). */
int pauli_add(const pauli_op *A, double alpha_re, double alpha_im, const pauli_op *B,
              double beta_re, double beta_im, const pauli_trunc *t, pauli_op *out,
              pauli_ws *ws, void *stream);

/* out = trunc(in) (trim / cutoff of the Methods section). */
int pauli_truncate(const pauli_op *in, const pauli_trunc *t, pauli_op *out, pauli_ws *ws,
                   void *stream);

/* out = in / b for a finite real b != 0: every coefficient's parts divided
 * by b (IEEE division in FP64; FP32 outputs rounded once), exact zeros
 * (underflow) dropped, canonical order (the Krylov section's O'_n / b_n as a
 * call of its own).  `in` needs unique strings; PAULI_EINVAL for b = 0 or not
 * finite; PAULI_ECAPACITY as for pauli_add; its workspace is that of
 * PAULI_Q_TRUNCATE with no truncation. */
int pauli_divide(const pauli_op *in, double b, pauli_op *out, pauli_ws *ws, void *stream);

/* out = canonical form of in: duplicate strings summed in input order, exact
 * zeros dropped, library order.  Duplicates allowed; up to 2^28 strings. */
int pauli_canonicalize(const pauli_op *in, pauli_op *out, pauli_ws *ws, void *stream);

/* Depolarizing noise in place (Heisenberg time evolution section: a string
 * of length w is transmitted with rate exp(-eps w); one step of the noisy
 * evolution applies lambda = eps dt): every coefficient is multiplied by
 * f[w] = exp(-lambda w), the table computed on the host in double, w =
 * sites with x or z set.  FP32 coefficients are scaled in double and rounded
 * once.  A coefficient that underflows becomes an exact zero in place (the
 * next pauli_truncate drops it).  lambda >= 0, else PAULI_EINVAL.
 * Asynchronous on `stream`. */
int pauli_add_noise(pauli_op *A, double lambda, void *stream);

/* A <- A^dagger in place.  Every Pauli string is Hermitian, so the adjoint
 * of sum_k c_k P_k is sum_k conj(c_k) P_k: the imaginary part of every
 * coefficient changes sign; strings, order and size are unchanged (the
 * Heisenberg section's dagger, as in Tr(O(t) O0^dagger)).  Asynchronous on
 * `stream`. */
int pauli_dagger(pauli_op *A, void *stream);

/* out[2q] + i out[2q+1] (host, 2 Q->size doubles) = the coefficient in A of the
 * string q of Q, 0 when A lacks it.  A must be canonical (distinct strings in
 * canonical order, as every call of this library leaves it); Q's strings are
 * any.  With Q = {Z_j} and A = Z_i(t) this reads the two-point correlators
 * S_{i-j}(t) = Tr[Z_i(t) Z_j(0)]/2^N of the noisy-evolution results.
 * Synchronous at return. */
int pauli_coefficients(const pauli_op *A, const pauli_op *Q, double *out, pauli_ws *ws,
                       void *stream);

/* Order keys: for every string of A its 2W-word key whose ascending
 * lexicographic order (word 0 most significant, unsigned) is the library's
 * canonical storage order.  The key is a bijective mix of the string's x and
 * z words (two Feistel rounds with the MurmurHash3 fmix64 finalizer).  keys:
 * device array [A->size][2W], caller-owned.  Synchronous at return. */
int pauli_order_keys(const pauli_op *A, uint64_t *keys, void *stream);

/* Inverse of pauli_order_keys: the x and z words (word-major, capacity cap,
 * caller-owned device arrays) of n strings of n_qubits sites from their order
 * keys [n][2W].  The caller passes keys of n_qubits-site strings; bits beyond
 * n_qubits are returned as the inverse produces them.  Synchronous. */
int pauli_strings_from_order_keys(int32_t n_qubits, const uint64_t *keys, int64_t n,
                                  uint64_t *x, uint64_t *z, int64_t cap, void *stream);

/* One classical Runge-Kutta step of the Heisenberg equation dO/dt = i[H, O]
 * (Heisenberg time evolution section):
 *   k1 = i[H,O];  S2 = trunc(O + fl(dt/2) k1);  k2 = i[H,S2];
 *   S3 = trunc(O + fl(dt/2) k2);  k3 = i[H,S3];  S4 = trunc(O + dt k3);
 *   k4 = i[H,S4];  out = trunc((((O + c1 k1) + c2 k2) + c2 k3) + c1 k4),
 * c1 = fl(dt/6), c2 = fl(dt/3).  PAULI_C128 only. */
int pauli_rk4_step(const pauli_op *H, const pauli_op *O, double dt, const pauli_trunc *t,
                   pauli_op *out, pauli_ws *ws, void *stream);

/* One step of the Liouvillian Lanczos recursion (Krylov section, L = [H, .]):
 *   O'_n = [H, O_{n-1}] - b_{n-1} O_{n-2}    (O_prev = NULL at n = 1)
 *   b_n  = ||O'_n|| = sqrt(sum |c|^2)         (norm of the untruncated O'_n)
 *   O_n  = trunc(O'_n / b_n)                 (IEEE division per component)
 * *b_out (host) receives b_n.  On PAULI_BREAKDOWN O_next->size = 0.
 * For PAULI_C64K operators the commutator runs in FP32 with compensated sums
 * and everything after it in FP64 (O_n rounded to FP32).
 * flags: 0, or PAULI_REORTH_LOCAL: local re-orthogonalisation (not in the
 * paper, whose recursion is the three-term one; it is a no-op in exact
 * arithmetic without truncation): before b_n is taken, O'_n is replaced by
 *   O'_n - a_1 O_{n-1} - a_2 O_{n-2},   a_k = <O_k, O'_n> / <O_k, O_k>,
 * both coefficients computed from the same O'_n in FP64 (inner products and
 * norms summed in double-double and rounded once, then divided), the
 * combination summed as for pauli_add.  O_cur and O_prev must then be
 * canonical (PAULI_EINVAL otherwise); the workspace also holds O'_n in FP64. */
enum { PAULI_REORTH_LOCAL = 1 };
int pauli_lanczos_step(const pauli_op *H, const pauli_op *O_prev, const pauli_op *O_cur,
                       double b_prev, const pauli_trunc *t, uint32_t flags,
                       pauli_op *O_next, double *b_out, pauli_ws *ws, void *stream);

/* *out (host) = sum_k fl(fl(re_k^2) + fl(im_k^2)) (the squared Frobenius norm
 * Tr(A^dagger A)/2^N), double-double accumulation rounded once. */
int pauli_norm2(const pauli_op *A, double *out, pauli_ws *ws, void *stream);

/* out[0] + i out[1] (host) = <A, B> = Tr(A^dagger B)/2^N = sum over common
 * strings of conj(a) b.  B must be canonical. */
int pauli_inner(const pauli_op *A, const pauli_op *B, double out[2], pauli_ws *ws,
                void *stream);

/* S = <O0, O>/<O0, O0> = sum over common strings of conj(c0) c / sum |c0|^2
 * (out[0] + i out[1], host): the autocorrelation of the Heisenberg section,
 * which for unit O0 equals Tr(O(t) O0)/2^N.  O0 must be canonical and
 * nonzero (PAULI_EINVAL otherwise).  Both sums in double-double, rounded
 * once, then divided.  Synchronous at return. */
int pauli_correlator(const pauli_op *O0, const pauli_op *O, double out[2], pauli_ws *ws,
                     void *stream);

/* Workspace and output sizing from the operand sizes alone (host only, no
 * device work; only n_qubits, dtype and size of the operands are read, so
 * their device pointers may be NULL).  The operands are those of the call:
 *   PAULI_Q_COMMUTATOR, PAULI_Q_MULTIPLY, PAULI_Q_COMMUTATOR_TS1D: A = H (H0), B = O
 *   PAULI_Q_ADD: A and B
 *   PAULI_Q_TRUNCATE, PAULI_Q_CANONICALIZE, PAULI_Q_CANONICALIZE_TS1D: B = in
 *   PAULI_Q_LANCZOS, PAULI_Q_LANCZOS_REORTH (flag PAULI_REORTH_LOCAL),
 *   PAULI_Q_LANCZOS_TS1D: A = H (H0), B = O_cur, C = O_prev (nullable)
 *   PAULI_Q_RK4: A = H, B = O
 *   PAULI_Q_REDUCTION (norm2, inner, trace, coefficients, correlator,
 *   norm2_ts1d): A, B (nullable)
 * t is the truncation the call will receive (nullable).
 * *ws_bytes: a workspace that holds the call when it emits at most the
 * records its sizes bound (|H| |O| pairs, N |H0| |O| for translation-
 * symmetric calls, plus the operator terms) and no hash bin holds more than
 * 1.5 times the mean plus the records one string can collect; a call beyond
 * that returns PAULI_EWORKSPACE with its exact need.  The bound is loose
 * where few pairs anticommute (the engine sizes the real call after
 * counting its records).
 * *out_capacity_upper: an output capacity that always suffices.
 * PAULI_EINVAL for an unknown op or missing operand. */
enum {
  PAULI_Q_COMMUTATOR = 0,
  PAULI_Q_MULTIPLY = 1,
  PAULI_Q_ADD = 2,
  PAULI_Q_TRUNCATE = 3,
  PAULI_Q_CANONICALIZE = 4,
  PAULI_Q_LANCZOS = 5,
  PAULI_Q_LANCZOS_REORTH = 6,
  PAULI_Q_RK4 = 7,
  PAULI_Q_COMMUTATOR_TS1D = 8,
  PAULI_Q_CANONICALIZE_TS1D = 9,
  PAULI_Q_LANCZOS_TS1D = 10,
  PAULI_Q_REDUCTION = 11
};
int pauli_workspace_query(int op, const pauli_op *A, const pauli_op *B, const pauli_op *C,
                          const pauli_trunc *t, size_t *ws_bytes, int64_t *out_capacity_upper);

/* ------------------------------------------------------------------------ */
/* b_n continuation network: a window of 16 Lanczos coefficients in, the next */
/* 16 out; 16 -> 256 -> 256 -> 16, GELU(x) = x (1 + erf(x/sqrt 2))/2 on the   */
/* hidden layers.  Every matrix product runs on the matrix cores with BF16    */
/* operands (round to nearest even) and FP32 accumulation; biases, GELU, the  */
/* loss and Adam run in FP32.  All pointers are device pointers owned by the   */
/* caller.  The flat parameter vector holds, in order: W1[256][16], b1[256],   */
/* W2[256][256], b2[256], W3[16][256], b3[16] (pauli_mlp_num_params() floats). */
/* ------------------------------------------------------------------------ */
typedef struct pauli_mlp {
  int32_t n_in, n_hidden, n_out; /* must be 16, 256, 16 */
  float *params;                 /* fp32 master weights */
  uint16_t *params_bf16;         /* bf16 copy used by the matrix products */
  float *grads;                  /* written by pauli_mlp_loss_grad */
  float *adam_m, *adam_v;        /* Adam moments (start at zero) */
} pauli_mlp;

int64_t pauli_mlp_num_params(void);
/* params_bf16 = bf16(params). */
int pauli_mlp_sync(const pauli_mlp *net, void *stream);
/* y[batch][16] = net(x[batch][16]); batch a positive multiple of 32. */
int pauli_mlp_forward(const pauli_mlp *net, const float *x, int64_t batch, float *y,
                      pauli_ws *ws, void *stream);
/* Masked mean-squared error L = sum mask (y - t)^2 / sum mask over the batch
 * (*loss, host) and its gradient with respect to every parameter (net->grads).
 * acts (nullable, device, batch * 2112 floats) receives the intermediate
 * tensors as FP32, in order: X_bf16[16], Z1[256], Y1_bf16[256], Z2[256],
 * Y2_bf16[256], Y[16], dY_bf16[16], dY2[256], dZ2_bf16[256], dY1[256],
 * dZ1_bf16[256] per row, each block batch-major. */
int pauli_mlp_loss_grad(const pauli_mlp *net, const float *x, const float *target,
                        const float *mask, int64_t batch, double *loss, float *acts,
                        pauli_ws *ws, void *stream);
/* One Adam step (step index t >= 1) from net->grads; refreshes params_bf16. */
int pauli_mlp_adam(const pauli_mlp *net, double lr, double beta1, double beta2, double eps,
                   int64_t t, void *stream);
/* Minibatch training with the fused step kernels: for every epoch e and
 * minibatch k (rows order[e n + k batch ...], batch rows, the last one of an
 * epoch shorter when batch does not divide n), one kernel runs the forward
 * pass, the masked MSE and the backward pass of 32 rows per block with the
 * activations in LDS and every product on the matrix cores (the BF16
 * operands and FP32 epilogues of pauli_mlp_loss_grad), a second sums the
 * blocks' gradient shares in block order and takes the Adam step (step
 * index t0 + 1, t0 + 2, ...).  x, t, mask: device [n][16]; order: device
 * int32 [epochs][n], each a permutation of 0..n-1 (not checked); losses:
 * device double [epochs][ceil(n / batch)] receives every minibatch's loss;
 * net->grads holds the last minibatch's gradient.  1 <= batch <= 4096.
 * Synchronous at return. */
int pauli_mlp_train(const pauli_mlp *net, const float *x, const float *t, const float *mask,
                    int64_t n, const int32_t *order, int64_t epochs, int32_t batch, double lr,
                    double beta1, double beta2, double eps, int64_t t0, double *losses,
                    pauli_ws *ws, void *stream);
/* C[M][N] (fp32) = A(M x K) B(K x N) with BF16 operands on the matrix cores;
 * A(m,k) = transA ? A[k*lda + m] : A[m*lda + k], B(k,n) = transB ? B[n*ldb + k]
 * : B[k*ldb + n]; M and N multiples of 16. */
int pauli_gemm_bf16(const uint16_t *A, int lda, int transA, const uint16_t *B, int ldb,
                    int transB, float *C, int ldc, int M, int N, int K, void *stream);

/* Counters of the last engine pass of this thread's last call (diagnostics and
 * the algorithmic byte counts of the benchmark). */
typedef struct pauli_stats {
  int64_t emitted;   /* records produced: anticommuting pairs + operator terms
                        (calls other than the Lanczos step leave out strings
                        above the length cap, which depends on the key alone) */
  int64_t unique;    /* distinct emitted strings with a nonzero merged coefficient */
  int64_t survivors; /* of those, left after the length and |c| filters */
  int64_t output;    /* strings written to the output */
  int32_t passes;    /* hash-range passes */
  int32_t buckets;   /* merge buckets */
  int32_t host_syncs; /* times the host waited for the stream (control-block
                         reads): one for a call planned from its sizes (at most
                         2^18 possible records, workspace for that bound), more
                         when the count must be read first or the top-M select
                         needs the host */
  int32_t reserved;
} pauli_stats;
void pauli_last_stats(pauli_stats *out);

/* Totals over every engine pass of this thread since the last reset (a
 * Runge-Kutta step makes eight passes, a Lanczos step one or two): strings
 * read as inputs, records emitted, merged strings, output strings, and the
 * algorithmic HBM bytes (inputs + 2 emitted + 2 merged + output) times the
 * record size (16 W + 16 bytes in FP64, 16 W + 8 in FP32) that the method
 * must move once its products are materialised.  reset != 0 clears them
 * after reading. */
typedef struct pauli_totals {
  int64_t calls;
  int64_t inputs;
  int64_t emitted;
  int64_t unique;
  int64_t output;
  double alg_bytes;
} pauli_totals;
void pauli_read_totals(pauli_totals *out, int reset);

/* Static description of the error code. */
const char *pauli_strerror(int status);
/* Text of the last HIP error seen by this thread (empty if none). */
const char *pauli_last_error(void);

/* Optional per-kernel timing with HIP events on the caller's stream.
 * pauli_profile_enable(1) clears the log and starts recording;
 * pauli_profile_read fills `buf` with one line per kernel name:
 * "name count total_ms\n" and returns the number of bytes needed.
 * pauli_profile_only("k_a,k_b") limits the events to the named kernels (each
 * timed kernel costs two event records on the stream); NULL or "" times every
 * kernel.  The filter stays until the next pauli_profile_only call. */
void pauli_profile_enable(int on);
void pauli_profile_only(const char *names);
size_t pauli_profile_read(char *buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* PAULI_H */
