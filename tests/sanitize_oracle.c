/* Sanitizer driver of the CPU oracle: builds seeded random operators and
 * runs every oracle routine on them (one and two mask words), so that an
 * AddressSanitizer / UndefinedBehaviorSanitizer build of pauli_oracle.c
 * reports any out-of-bounds access, leak or undefined operation.  Exit code
 * 0 when every call returned a valid status. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/pauli_oracle.h"

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint64_t next64(void) { /* xorshift64* */
  state ^= state >> 12;
  state ^= state << 25;
  state ^= state >> 27;
  return state * 0x2545F4914F6CDD1Dull;
}
static double unit(void) { return (double)(next64() >> 11) * (1.0 / 9007199254740992.0) - 0.5; }

/* canonical operator of (up to) n random strings on n_qubits sites, each
 * site occupied with probability 1/4 */
static or_op random_op(int n_qubits, int64_t n) {
  or_op raw, out;
  memset(&out, 0, sizeof(out));
  raw.n_qubits = n_qubits;
  raw.n = n;
  raw.x = calloc((size_t)(2 * n + 2), sizeof(uint64_t));
  raw.z = calloc((size_t)(2 * n + 2), sizeof(uint64_t));
  raw.re = calloc((size_t)(n + 1), sizeof(double));
  raw.im = calloc((size_t)(n + 1), sizeof(double));
  for (int64_t k = 0; k < n; k++) {
    for (int j = 0; j < n_qubits; j++) {
      const uint64_t r = next64();
      if ((r & 3) == 0) {
        const int p = 1 + (int)((r >> 2) % 3);
        if (p & 1) raw.x[2 * k + j / 64] |= 1ull << (j % 64);
        if (p & 2) raw.z[2 * k + j / 64] |= 1ull << (j % 64);
      }
    }
    raw.re[k] = unit();
    raw.im[k] = unit();
  }
  if (or_canonicalize(&raw, &out)) exit(2);
  or_free(&raw);
  return out;
}

static int fails = 0;
static void ok(int rc, const char *what) {
  if (rc != OR_OK && rc != OR_BREAKDOWN) {
    fprintf(stderr, "%s returned %d\n", what, rc);
    fails++;
  }
}

static void run(int n_qubits) {
  or_op H = random_op(n_qubits, 12), O = random_op(n_qubits, 80), P = random_op(n_qubits, 40);
  or_op a = {0}, b = {0}, c = {0}, d = {0}, e = {0}, f = {0}, g = {0}, h = {0}, k = {0};
  double re, im, bn;
  ok(or_commutator(&H, &O, OR_F64, &a), "commutator");
  ok(or_commutator(&H, &O, OR_F32K, &b), "commutator f32k");
  ok(or_product(&H, &P, &c), "product");
  ok(or_add(&a, 1.0, 0.5, &P, -0.25, 0.0, &d), "add");
  or_trunc t = {6, 1e-3, 20, &P};
  ok(or_truncate(&d, &t, &e), "truncate");
  ok(or_divide(&a, 3.0, &f), "divide");
  ok(or_add_noise(&a, 0.1, &g), "add_noise");
  or_inner(&a, &d, &re, &im);
  (void)or_norm2(&a);
  or_trunc tl = {0, 0.0, 50, NULL};
  ok(or_lanczos_step(&H, &P, &O, 0.7, &tl, OR_F64, &h, &bn), "lanczos");
  or_free(&h);
  ok(or_lanczos_step_reorth(&H, &P, &O, 0.7, &tl, OR_F32K, &h, &bn), "lanczos reorth");
  ok(or_rk4_step(&H, &O, 0.02, &tl, &k), "rk4");
  /* translation-symmetric operators: representatives of O, commutator, norm, step */
  or_op rep = {0}, ts = {0}, tsn = {0};
  rep.n_qubits = n_qubits;
  rep.n = O.n;
  rep.x = calloc((size_t)(2 * O.n + 2), sizeof(uint64_t));
  rep.z = calloc((size_t)(2 * O.n + 2), sizeof(uint64_t));
  rep.re = calloc((size_t)(O.n + 1), sizeof(double));
  rep.im = calloc((size_t)(O.n + 1), sizeof(double));
  for (int64_t q = 0; q < O.n; q++) {
    (void)or_ts_canonical(n_qubits, &O.x[2 * q], &O.z[2 * q], &rep.x[2 * q], &rep.z[2 * q]);
    rep.re[q] = O.re[q];
    rep.im[q] = O.im[q];
  }
  or_op repc = {0};
  ok(or_canonicalize(&rep, &repc), "canonicalize representatives");
  ok(or_commutator_ts(&H, &repc, &ts), "commutator_ts");
  (void)or_norm2_ts(&ts);
  ok(or_lanczos_step_ts(&H, NULL, &repc, 0.0, &tl, &tsn, &bn), "lanczos_ts");
  or_op *all[] = {&H, &O, &P, &a, &b, &c, &d, &e, &f, &g, &h, &k, &rep, &repc, &ts, &tsn};
  for (size_t q = 0; q < sizeof(all) / sizeof(all[0]); q++) or_free(all[q]);
}

int main(void) {
  run(20);
  run(100);
  double v[5] = {1e300, -1e300, 1.0, 1e-300, -1.0};
  if (or_exact_sum(v, 5) != 1e-300) fails++;
  if (fails) return 1;
  printf("sanitizer driver ok\n");
  return 0;
}
