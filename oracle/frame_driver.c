/*
 * Stand-alone driver of the frame oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Built together with frame.c into an executable (with AddressSanitizer and
 * UndefinedBehaviorSanitizer by the CPU test suite), it reads one circuit
 * from standard input and prints the frame size, the norm of the amplitudes
 * and the measurement outcomes, so that the oracle's memory handling can be
 * checked on circuits of every word count.  With the argument "multi" (or
 * "general") the circuit runs on the multiframe simulation (basic COALESCE,
 * or COALESCE through the basis circuit) and the element count, norm and
 * outcomes are summed over its frames, followed by the number of frames and
 * whether they are pairwise orthogonal.
 *
 * Input: "n seed", then n basis bits, then the gate count G, then G lines
 * "op q0 q1 q2 num den" (the gate codes of frame.c).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void *ofr_new(int n, const uint8_t *init_bits, uint64_t seed);
void ofr_free(void *F);
int ofr_apply(void *F, int op, int q0, int q1, int q2, int64_t num, int64_t den);
size_t ofr_size(void *F);
int ofr_fragile(void *F);
size_t ofr_outcomes(void *F, uint8_t *out, size_t cap);
size_t ofr_read(void *F, uint64_t *tableau, uint64_t *sigma, double *amp, size_t cap);
void *omf_new(int n, const uint8_t *init_bits, uint64_t seed);
void omf_free(void *M);
int omf_apply(void *M, int op, int q0, int q1, int q2, int64_t num, int64_t den);
size_t omf_nframes(void *M);
size_t omf_frame_size(void *M, size_t i);
size_t omf_read(void *M, size_t i, uint64_t *tableau, uint64_t *sigma, double *amp, size_t cap);
int omf_fragile(void *M);
int omf_orthogonal(void *M);
size_t omf_outcomes(void *M, uint8_t *out, size_t cap);
void omf_set_general(void *M, int general);

static int run_multi(int n, const uint8_t *bits, uint64_t seed, int general) {
  void *M = omf_new(n, bits, seed);
  if (!M) return 2;
  omf_set_general(M, general);
  long G;
  if (scanf("%ld", &G) != 1 || G < 0) return 2;
  for (long g = 0; g < G; ++g) {
    int op, q0, q1, q2;
    long long num, den;
    if (scanf("%d %d %d %d %lld %lld", &op, &q0, &q1, &q2, &num, &den) != 6) return 2;
    if (omf_apply(M, op, q0, q1, q2, (int64_t)num, (int64_t)den) < 0) return 3;
  }
  const int W = (n + 63) / 64;
  const size_t nf = omf_nframes(M);
  size_t K = 0;
  double norm = 0;
  uint64_t *tab = malloc((size_t)n * 2 * W * 8);
  for (size_t i = 0; i < nf; ++i) {
    const size_t k = omf_frame_size(M, i);
    uint64_t *sig = malloc((k ? k : 1) * W * 8);
    double *amp = malloc((k ? k : 1) * 2 * sizeof(double));
    omf_read(M, i, tab, sig, amp, k);
    for (size_t j = 0; j < k; ++j) norm += amp[2 * j] * amp[2 * j] + amp[2 * j + 1] * amp[2 * j + 1];
    K += k;
    free(amp);
    free(sig);
  }
  size_t m = omf_outcomes(M, NULL, 0);
  uint8_t *out = malloc(m ? m : 1);
  omf_outcomes(M, out, m);
  printf("K %zu\nnorm %.17g\nfragile %d\noutcomes", K, norm, omf_fragile(M));
  for (size_t i = 0; i < m; ++i) printf(" %d", out[i]);
  printf("\nframes %zu\northogonal %d\n", nf, omf_orthogonal(M));
  free(out);
  free(tab);
  omf_free(M);
  return 0;
}

int main(int argc, char **argv) {
  const int multi = argc > 1 && (!strcmp(argv[1], "multi") || !strcmp(argv[1], "general"));
  const int general = argc > 1 && !strcmp(argv[1], "general");
  int n;
  unsigned long long seed;
  if (scanf("%d %llu", &n, &seed) != 2 || n < 1 || n > 512) return 2;
  uint8_t *bits = calloc((size_t)n, 1);
  for (int q = 0; q < n; ++q) {
    int b;
    if (scanf("%d", &b) != 1) return 2;
    bits[q] = (uint8_t)(b & 1);
  }
  if (multi) {
    const int rc = run_multi(n, bits, (uint64_t)seed, general);
    free(bits);
    return rc;
  }
  void *F = ofr_new(n, bits, (uint64_t)seed);
  if (!F) return 2;
  long G;
  if (scanf("%ld", &G) != 1 || G < 0) return 2;
  for (long g = 0; g < G; ++g) {
    int op, q0, q1, q2;
    long long num, den;
    if (scanf("%d %d %d %d %lld %lld", &op, &q0, &q1, &q2, &num, &den) != 6) return 2;
    if (ofr_apply(F, op, q0, q1, q2, (int64_t)num, (int64_t)den) < 0) return 3;
  }
  size_t K = ofr_size(F);
  int W = (n + 63) / 64;
  uint64_t *tab = malloc((size_t)n * 2 * W * 8);
  uint64_t *sig = malloc((K ? K : 1) * W * 8);
  double *amp = malloc((K ? K : 1) * 2 * sizeof(double));
  ofr_read(F, tab, sig, amp, K);
  double norm = 0;
  for (size_t j = 0; j < K; ++j) norm += amp[2 * j] * amp[2 * j] + amp[2 * j + 1] * amp[2 * j + 1];
  size_t m = ofr_outcomes(F, NULL, 0);
  uint8_t *out = malloc(m ? m : 1);
  ofr_outcomes(F, out, m);
  printf("K %zu\nnorm %.17g\nfragile %d\noutcomes", K, norm, ofr_fragile(F));
  for (size_t i = 0; i < m; ++i) printf(" %d", out[i]);
  printf("\n");
  free(out); free(amp); free(sig); free(tab); free(bits);
  ofr_free(F);
  return 0;
}
