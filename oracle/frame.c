/*
 * Stabilizer-frame oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, single-threaded CPU implementation of single-frame simulation from
 * Garcia & Markov, "Simulation of Quantum Circuits via Stabilizer Frames":
 * a stabilizer matrix kept in row-reduced echelon form (Invariant 1) plus a
 * sorted list of (phase vector, complex amplitude) pairs (Definition 1).
 * Only tests, the smoke check and the bench's CPU-baseline leg may load it;
 * the HIP library never does, and the two share no code.
 *
 * Conventions (readings of the paper where it leaves the choice open):
 *  - Pauli literal bits: (x,z) = 00 I, 01 Z, 10 X, 11 Y (section 2.2).
 *    A row with bits (x,z) and sign bit s is (-1)^s (x) literals.
 *  - Canonical form: fully reduced row echelon form of the n x 2n bit matrix
 *    with column order x_0..x_{n-1}, z_0..z_{n-1}; rows sorted by pivot, so the
 *    X-block comes first (Figure 2b caption).
 *  - Qubit 0 is the most significant bit of a basis index; bit q of a packed
 *    vector is word q>>6, bit q&63.
 *  - Phase vector bit i is the sign of canonical row i (1 means -1).
 *  - The canonical stabilizer state psi(M,sigma) has a real positive amplitude
 *    at b*, the smallest basis string in its support.
 *  - Canonical order of elements: ascending sum_i sigma_i 2^i.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

enum { OP_H, OP_S, OP_SDG, OP_X, OP_Y, OP_Z, OP_CNOT, OP_CZ, OP_T, OP_TDG,
       OP_PHASE, OP_CPHASE, OP_TOF, OP_MEASURE, OP_CPHASE_D, OP_TOF_D };

#define PRUNE_EPS 1e-12
#define FRAGILE_AMP 1e-9
#define FRAGILE_COIN 1e-12

typedef struct { double re, im; } cplx;

static cplx cmul(cplx a, cplx b) {
  cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
  return r;
}
static cplx cadd(cplx a, cplx b) { cplx r = {a.re + b.re, a.im + b.im}; return r; }
static cplx cscale(cplx a, double s) { cplx r = {a.re * s, a.im * s}; return r; }
/* i^e for e mod 4 */
static cplx ipow(int e) {
  static const cplx tab[4] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
  return tab[((e % 4) + 4) % 4];
}

static int getbit(const uint64_t *v, int q) { return (int)((v[q >> 6] >> (q & 63)) & 1u); }
static void setbit(uint64_t *v, int q, int b) {
  uint64_t m = (uint64_t)1 << (q & 63);
  if (b) v[q >> 6] |= m; else v[q >> 6] &= ~m;
}
static void flipbit(uint64_t *v, int q) { v[q >> 6] ^= (uint64_t)1 << (q & 63); }
static int parity_and(const uint64_t *a, const uint64_t *b, int W) {
  uint64_t acc = 0;
  for (int w = 0; w < W; ++w) acc ^= a[w] & b[w];
  return __builtin_parityll(acc);
}
static int popcount_and(const uint64_t *a, const uint64_t *b, int W) {
  int c = 0;
  for (int w = 0; w < W; ++w) c += __builtin_popcountll(a[w] & b[w]);
  return c;
}

/* Table 1: exponent e of i in (literal 1)(literal 2) = i^e (literal 1*2).
 * XY = iZ, YZ = iX, ZX = iY and the reversed products carry -i. */
static int pauli_g(int x1, int z1, int x2, int z2) {
  if (!x1 && !z1) return 0;
  if (x1 && z1) return z2 - x2;              /* Y * . */
  if (x1 && !z1) return z2 * (2 * x2 - 1);    /* X * . */
  return x2 * (1 - 2 * z2);                   /* Z * . */
}

/* ------------------------------------------------------------------------- */
/* Stabilizer matrix without signs (signs live in each phase vector).         */
/* ------------------------------------------------------------------------- */
typedef struct {
  int n, W;
  uint64_t *x, *z; /* n rows of W words */
} tab_t;

static uint64_t *RX(tab_t *t, int i) { return t->x + (size_t)i * t->W; }
static uint64_t *RZ(tab_t *t, int i) { return t->z + (size_t)i * t->W; }

static void tab_init(tab_t *t, int n) {
  t->n = n; t->W = (n + 63) / 64;
  t->x = calloc((size_t)n * t->W, 8);
  t->z = calloc((size_t)n * t->W, 8);
}
static void tab_free(tab_t *t) { free(t->x); free(t->z); t->x = t->z = NULL; }
static void tab_copy(tab_t *dst, const tab_t *src) {
  tab_init(dst, src->n);
  memcpy(dst->x, src->x, (size_t)src->n * src->W * 8);
  memcpy(dst->z, src->z, (size_t)src->n * src->W * 8);
}

/* sign bit c of the product row_i * row_k of two commuting unsigned rows:
 * row_i row_k = (-1)^c (row_i xor row_k) (section 2.2, Table 1). */
static int rowprod_sign(tab_t *t, int i, int k) {
  int e = 0;
  for (int q = 0; q < t->n; ++q)
    e += pauli_g(getbit(RX(t, i), q), getbit(RZ(t, i), q), getbit(RX(t, k), q), getbit(RZ(t, k), q));
  e = ((e % 4) + 4) % 4;
  if (e & 1) { fprintf(stderr, "oracle: rows %d,%d anticommute\n", i, k); abort(); }
  return e >> 1;
}

/* Row operations recorded while the matrix is changed, replayed on every
 * phase vector (memoised row updates, section 3). */
typedef struct { int kind, i, k, c; } rowop; /* kind 0: swap i,k ; 1: sigma_i ^= sigma_k ^ c */
typedef struct { rowop *op; size_t len, cap; } oplog;

static void log_push(oplog *L, int kind, int i, int k, int c) {
  if (L->len == L->cap) { L->cap = L->cap ? 2 * L->cap : 64; L->op = realloc(L->op, L->cap * sizeof(rowop)); }
  L->op[L->len].kind = kind; L->op[L->len].i = i; L->op[L->len].k = k; L->op[L->len].c = c;
  L->len++;
}

static void row_swap(tab_t *t, int i, int k, oplog *L) {
  if (i == k) return;
  for (int w = 0; w < t->W; ++w) {
    uint64_t a = RX(t, i)[w]; RX(t, i)[w] = RX(t, k)[w]; RX(t, k)[w] = a;
    a = RZ(t, i)[w]; RZ(t, i)[w] = RZ(t, k)[w]; RZ(t, k)[w] = a;
  }
  log_push(L, 0, i, k, 0);
}
/* row_i <- row_i * row_k */
static void row_mul(tab_t *t, int i, int k, oplog *L) {
  int c = rowprod_sign(t, i, k);
  for (int w = 0; w < t->W; ++w) { RX(t, i)[w] ^= RX(t, k)[w]; RZ(t, i)[w] ^= RZ(t, k)[w]; }
  log_push(L, 1, i, k, c);
}

static int colbit(tab_t *t, int row, int col) {
  return col < t->n ? getbit(RX(t, row), col) : getbit(RZ(t, row), col - t->n);
}

/* Gaussian elimination to the canonical (fully reduced) row echelon form. */
static void canonicalize(tab_t *t, oplog *L) {
  int r = 0;
  for (int col = 0; col < 2 * t->n && r < t->n; ++col) {
    int piv = -1;
    for (int i = r; i < t->n; ++i) if (colbit(t, i, col)) { piv = i; break; }
    if (piv < 0) continue;
    row_swap(t, r, piv, L);
    for (int i = 0; i < t->n; ++i)
      if (i != r && colbit(t, i, col)) row_mul(t, i, r, L);
    ++r;
  }
  if (r != t->n) { fprintf(stderr, "oracle: tableau lost rank\n"); abort(); }
}

static void replay(const oplog *L, uint64_t *sig) {
  for (size_t j = 0; j < L->len; ++j) {
    const rowop *o = &L->op[j];
    if (o->kind == 0) {
      int a = getbit(sig, o->i), b = getbit(sig, o->k);
      setbit(sig, o->i, b); setbit(sig, o->k, a);
    } else {
      if (getbit(sig, o->k) ^ o->c) flipbit(sig, o->i);
    }
  }
}

/* number of X-block rows of a canonical matrix */
static int xblock(tab_t *t) {
  int k = 0;
  for (int i = 0; i < t->n; ++i) {
    int any = 0;
    for (int w = 0; w < t->W; ++w) any |= RX(t, i)[w] != 0;
    if (!any) break;
    k = i + 1;
  }
  return k;
}
static int lowest_bit(const uint64_t *v, int W) {
  for (int w = 0; w < W; ++w) if (v[w]) return 64 * w + __builtin_ctzll(v[w]);
  return -1;
}

/* ------------------------------------------------------------------------- */
/* b*(sigma): the unique b with b[p_l] = 0 on every X-block pivot and         */
/* z_h . b = sigma_h on every Z-block row h (Observation 1: the generators    */
/* are a linear system whose solutions are the support).  b* depends linearly */
/* on the Z-block signs; beta[h] is the solution for sigma = e_h.             */
/* ------------------------------------------------------------------------- */
typedef struct {
  int n, W, k;
  int *piv;        /* X-block pivots p_l, l < k */
  uint64_t *beta;  /* n rows (only h >= k used) of W words */
} bmap_t;

static void bmap_build(bmap_t *B, tab_t *t) {
  int n = t->n, W = t->W;
  B->n = n; B->W = W; B->k = xblock(t);
  B->piv = malloc(sizeof(int) * (n ? n : 1));
  for (int l = 0; l < B->k; ++l) B->piv[l] = lowest_bit(RX(t, l), W);
  /* constraint matrix E (n x n) augmented with the identity; invert. */
  uint64_t *E = calloc((size_t)n * W, 8), *I = calloc((size_t)n * W, 8);
  for (int r = 0; r < n; ++r) {
    if (r < B->k) setbit(E + (size_t)r * W, B->piv[r], 1);
    else memcpy(E + (size_t)r * W, RZ(t, r), W * 8);
    setbit(I + (size_t)r * W, r, 1);
  }
  for (int col = 0; col < n; ++col) {
    int p = -1;
    for (int r = col; r < n; ++r) if (getbit(E + (size_t)r * W, col)) { p = r; break; }
    if (p < 0) { fprintf(stderr, "oracle: singular support system\n"); abort(); }
    for (int w = 0; w < W; ++w) {
      uint64_t a = E[(size_t)p * W + w]; E[(size_t)p * W + w] = E[(size_t)col * W + w]; E[(size_t)col * W + w] = a;
      a = I[(size_t)p * W + w]; I[(size_t)p * W + w] = I[(size_t)col * W + w]; I[(size_t)col * W + w] = a;
    }
    for (int r = 0; r < n; ++r)
      if (r != col && getbit(E + (size_t)r * W, col))
        for (int w = 0; w < W; ++w) { E[(size_t)r * W + w] ^= E[(size_t)col * W + w]; I[(size_t)r * W + w] ^= I[(size_t)col * W + w]; }
  }
  /* E^{-1} = I (rows).  beta[h] = column h of E^{-1}. */
  B->beta = calloc((size_t)n * W, 8);
  for (int r = 0; r < n; ++r)
    for (int h = 0; h < n; ++h)
      if (getbit(I + (size_t)r * W, h)) setbit(B->beta + (size_t)h * W, r, 1);
  free(E); free(I);
}
static void bmap_free(bmap_t *B) { free(B->piv); free(B->beta); }

static void bstar(const bmap_t *B, const uint64_t *sig, uint64_t *out) {
  memset(out, 0, B->W * 8);
  for (int h = B->k; h < B->n; ++h)
    if (getbit(sig, h))
      for (int w = 0; w < B->W; ++w) out[w] ^= B->beta[(size_t)h * B->W + w];
}

/* Amplitude of psi(M,sigma) at basis string b, as 2^{-k/2} * u with |u| = 1;
 * returns 0 when b is outside the support.  psi is proportional to
 * prod_l (I + g_l)/2 |b*>, so the amplitude at b* ^ x_S is the phase picked up
 * by applying the X-block generators in S to |b*>. */
static int amp_at(tab_t *t, const bmap_t *B, const uint64_t *sig, const uint64_t *bst,
                  const uint64_t *b, cplx *u) {
  int W = t->W, e = 0;
  uint64_t v[8];
  memcpy(v, bst, W * 8);
  for (int l = 0; l < B->k; ++l) {
    if (!getbit(b, B->piv[l])) continue;
    /* g|v> = (-1)^{s + z.v} i^{|x&z|} |v ^ x> */
    e += 2 * (getbit(sig, l) ^ parity_and(RZ(t, l), v, W)) + popcount_and(RX(t, l), RZ(t, l), W);
    for (int w = 0; w < W; ++w) v[w] ^= RX(t, l)[w];
  }
  for (int w = 0; w < W; ++w) if (v[w] != b[w]) return 0;
  *u = ipow(e);
  return 1;
}

/* ------------------------------------------------------------------------- */
/* Frame                                                                      */
/* ------------------------------------------------------------------------- */
typedef struct {
  tab_t t;
  int n, W;
  size_t K, cap;
  uint64_t *sig; /* K x W */
  cplx *amp;
  uint64_t seed, nmeas;
  uint8_t *out; size_t nout, outcap;
  int fragile;
} frame_t;

static uint64_t *SIG(frame_t *F, size_t j) { return F->sig + j * F->W; }

static void frame_reserve(frame_t *F, size_t K) {
  if (K <= F->cap) return;
  size_t c = F->cap ? F->cap : 16;
  while (c < K) c *= 2;
  F->sig = realloc(F->sig, c * F->W * 8);
  F->amp = realloc(F->amp, c * sizeof(cplx));
  F->cap = c;
}

static int sig_cmp_W;
static int elem_cmp(const void *a, const void *b) {
  const uint64_t *x = a, *y = b;
  for (int w = sig_cmp_W - 1; w >= 0; --w) {
    if (x[w] < y[w]) return -1;
    if (x[w] > y[w]) return 1;
  }
  return 0;
}

/* Sort by sigma, sum amplitudes of equal sigma, drop |a| <= eps. */
static void frame_merge(frame_t *F) {
  int W = F->W;
  size_t rec = (size_t)W * 8 + sizeof(cplx);
  unsigned char *buf = malloc(rec * (F->K ? F->K : 1));
  for (size_t j = 0; j < F->K; ++j) {
    memcpy(buf + j * rec, SIG(F, j), W * 8);
    memcpy(buf + j * rec + W * 8, &F->amp[j], sizeof(cplx));
  }
  sig_cmp_W = W;
  qsort(buf, F->K, rec, elem_cmp);
  size_t out = 0;
  for (size_t j = 0; j < F->K;) {
    size_t e = j + 1;
    cplx s;
    memcpy(&s, buf + j * rec + W * 8, sizeof(cplx));
    while (e < F->K && elem_cmp(buf + e * rec, buf + j * rec) == 0) {
      cplx a; memcpy(&a, buf + e * rec + W * 8, sizeof(cplx));
      s = cadd(s, a); ++e;
    }
    double mag = sqrt(s.re * s.re + s.im * s.im);
    if (mag > PRUNE_EPS) {
      if (mag < FRAGILE_AMP) F->fragile = 1;
      memcpy(SIG(F, out), buf + j * rec, W * 8);
      F->amp[out] = s;
      ++out;
    }
    j = e;
  }
  F->K = out;
  free(buf);
}

static void frame_sort(frame_t *F) { frame_merge(F); }

/* ------------------------------------------------------------------------- */
/* Clifford gates: Table 2 conjugation rules and the sign flip they put on    */
/* each row.                                                                  */
/* ------------------------------------------------------------------------- */
static void clifford_columns(tab_t *t, int op, int a, int b, uint64_t *f) {
  int W = t->W;
  memset(f, 0, W * 8);
  for (int i = 0; i < t->n; ++i) {
    uint64_t *x = RX(t, i), *z = RZ(t, i);
    int xa = getbit(x, a), za = getbit(z, a), flip = 0;
    switch (op) {
      case OP_H: flip = xa & za; setbit(x, a, za); setbit(z, a, xa); break;  /* X->Z, Y->-Y, Z->X */
      case OP_S: flip = xa & za; setbit(z, a, za ^ xa); break;               /* X->Y, Y->-X */
      case OP_SDG: flip = xa & !za; setbit(z, a, za ^ xa); break;            /* X->-Y, Y->X */
      case OP_X: flip = za; break;
      case OP_Z: flip = xa; break;
      case OP_Y: flip = xa ^ za; break;
      case OP_CNOT: {
        int xb = getbit(x, b), zb = getbit(z, b);
        flip = xa & zb & (xb ^ za ^ 1);
        setbit(x, b, xb ^ xa); setbit(z, a, za ^ zb);
        break;
      }
      case OP_CZ: {
        int xb = getbit(x, b), zb = getbit(z, b);
        flip = xa & xb & (za ^ zb);
        setbit(z, a, za ^ xb); setbit(z, b, zb ^ xa);
        break;
      }
      default: abort();
    }
    if (flip) setbit(f, i, 1);
  }
}

/* Row b' of the gate matrix: U[b', b] for the (at most two) b with a non-zero
 * entry.  Returns the count. */
static int gate_row(int op, int a, int c2, const uint64_t *bp, int W, uint64_t bs[2][8], cplx coef[2]) {
  for (int j = 0; j < 2; ++j) memcpy(bs[j], bp, W * 8);
  int ba = getbit(bp, a);
  const double r2 = 0.70710678118654752440;
  switch (op) {
    case OP_H:
      setbit(bs[0], a, 0); setbit(bs[1], a, 1);
      coef[0].re = r2; coef[0].im = 0;
      coef[1].re = ba ? -r2 : r2; coef[1].im = 0;
      return 2;
    case OP_S: coef[0] = ipow(ba); return 1;
    case OP_SDG: coef[0] = ipow(-ba); return 1;
    case OP_X: flipbit(bs[0], a); coef[0] = ipow(0); return 1;
    case OP_Z: coef[0] = ipow(2 * ba); return 1;
    case OP_Y: /* Y|0> = i|1>, Y|1> = -i|0>: source bit is 1 - ba */
      flipbit(bs[0], a); coef[0] = ipow(ba ? 1 : 3); return 1;
    case OP_CNOT: if (getbit(bp, a)) flipbit(bs[0], c2); coef[0] = ipow(0); return 1;
    case OP_CZ: coef[0] = ipow(2 * (ba & getbit(bp, c2))); return 1;
  }
  abort();
}

/* ROTATE(F, U) with global-phase maintenance (section 3). */
static void frame_clifford(frame_t *F, int op, int a, int b) {
  int W = F->W;
  tab_t old; tab_copy(&old, &F->t);
  bmap_t Bo; bmap_build(&Bo, &old);
  uint64_t f[8];
  clifford_columns(&F->t, op, a, b, f);
  oplog L = {0};
  canonicalize(&F->t, &L);
  bmap_t Bn; bmap_build(&Bn, &F->t);
  double scale = ldexp(1.0, 0);
  int dk = Bn.k - Bo.k; /* 2^{(k'-k)/2} */
  if (dk == 1) scale = sqrt(2.0); else if (dk == -1) scale = sqrt(0.5); else if (dk != 0) abort();
  uint64_t so[8], sn[8], bo[8], bn[8], bs[2][8];
  cplx coef[2];
  for (size_t j = 0; j < F->K; ++j) {
    memcpy(so, SIG(F, j), W * 8);
    for (int w = 0; w < W; ++w) sn[w] = so[w] ^ f[w];
    replay(&L, sn);
    bstar(&Bo, so, bo);
    bstar(&Bn, sn, bn);
    int m = gate_row(op, a, b, bn, W, bs, coef);
    cplx om = {0, 0};
    for (int r = 0; r < m; ++r) {
      cplx u;
      if (amp_at(&old, &Bo, so, bo, bs[r], &u)) om = cadd(om, cmul(coef[r], u));
    }
    om = cscale(om, scale);
    double mag = sqrt(om.re * om.re + om.im * om.im);
    if (fabs(mag - 1.0) > 1e-9) { fprintf(stderr, "oracle: |omega| = %g\n", mag); abort(); }
    F->amp[j] = cmul(F->amp[j], om);
    memcpy(SIG(F, j), sn, W * 8);
  }
  frame_sort(F);
  free(L.op); bmap_free(&Bo); bmap_free(&Bn); tab_free(&old);
}

/* Z-block rows whose product is Z_q (q deterministic): greedy elimination on
 * the reduced Z-block.  Returns 0 if q is random. */
static int zq_rows(tab_t *t, int q, uint64_t *mask) {
  int W = t->W, k = xblock(t);
  for (int l = 0; l < k; ++l) if (getbit(RX(t, l), q)) return 0;
  uint64_t tgt[8] = {0};
  setbit(tgt, q, 1);
  memset(mask, 0, W * 8);
  for (int h = k; h < t->n; ++h) {
    int p = lowest_bit(RZ(t, h), W);
    if (getbit(tgt, p)) {
      for (int w = 0; w < W; ++w) tgt[w] ^= RZ(t, h)[w];
      setbit(mask, h, 1);
    }
  }
  for (int w = 0; w < W; ++w) if (tgt[w]) { fprintf(stderr, "oracle: Z_q not in group\n"); abort(); }
  return 1;
}

/* COFACTOR(F, q) (section 3) with the phase exp(i theta) put on the
 * |1>-cofactor; theta = 0 gives the plain cofactor used by measurement.
 * Returns 1 if the frame was split. */
static int frame_cofactor(frame_t *F, int q, cplx ph1, int apply_phase) {
  int W = F->W;
  uint64_t rq[8];
  if (zq_rows(&F->t, q, rq)) {
    /* deterministic: qubit value of each element is the parity of its signs
     * on the rows whose product is Z_q. */
    if (apply_phase)
      for (size_t j = 0; j < F->K; ++j)
        if (parity_and(SIG(F, j), rq, W)) F->amp[j] = cmul(F->amp[j], ph1);
    return 0;
  }
  tab_t old; tab_copy(&old, &F->t);
  bmap_t Bo; bmap_build(&Bo, &old);
  int k = Bo.k, p = -1;
  for (int l = 0; l < k; ++l) if (getbit(RX(&F->t, l), q)) p = l; /* highest X-row with X/Y at q */
  oplog L1 = {0}, L2 = {0};
  for (int i = 0; i < F->n; ++i)
    if (i != p && getbit(RX(&F->t, i), q)) row_mul(&F->t, i, p, &L1);
  memset(RX(&F->t, p), 0, W * 8);
  memset(RZ(&F->t, p), 0, W * 8);
  setbit(RZ(&F->t, p), q, 1);
  canonicalize(&F->t, &L2);
  bmap_t Bn; bmap_build(&Bn, &F->t);
  if (Bn.k != k - 1) abort();
  size_t K = F->K;
  frame_reserve(F, 2 * K);
  const double r2 = 0.70710678118654752440;
  uint64_t so[8], s1[8], sc[8], bo[8], bn[8];
  for (size_t j = K; j-- > 0;) {
    memcpy(so, SIG(F, j), W * 8);
    cplx a = F->amp[j];
    memcpy(s1, so, W * 8);
    replay(&L1, s1);
    bstar(&Bo, so, bo);
    for (int x = 0; x < 2; ++x) {
      memcpy(sc, s1, W * 8);
      setbit(sc, p, x);      /* row p is now (-1)^x Z_q */
      replay(&L2, sc);
      bstar(&Bn, sc, bn);
      cplx u;
      if (!amp_at(&old, &Bo, so, bo, bn, &u)) { fprintf(stderr, "oracle: child b* outside parent support\n"); abort(); }
      cplx c = cscale(cmul(a, u), r2);
      if (x == 1 && apply_phase) c = cmul(c, ph1);
      size_t dst = x ? K + j : j;
      memcpy(SIG(F, dst), sc, W * 8);
      F->amp[dst] = c;
    }
  }
  F->K = 2 * K;
  frame_merge(F);
  free(L1.op); free(L2.op); bmap_free(&Bo); bmap_free(&Bn); tab_free(&old);
  return 1;
}

/* A Pauli gate (X, Y or Z on qubit a) applied only to the elements whose
 * qubits with Z-row products m1 and m2 both read 1 (both qubits must be
 * deterministic).  A Pauli leaves the unsigned matrix as it is, so each
 * selected element gets the five-step factor of the gate and its sign flips;
 * the others are unchanged.  Used by the direct Toffoli (Eq. 2). */
static void frame_pauli_masked(frame_t *F, int op, int a, const uint64_t *m1, const uint64_t *m2) {
  int W = F->W;
  if (op != OP_X && op != OP_Y && op != OP_Z) abort();
  tab_t t2; tab_copy(&t2, &F->t);
  uint64_t f[8];
  clifford_columns(&t2, op, a, 0, f);
  tab_free(&t2);
  bmap_t B; bmap_build(&B, &F->t);
  uint64_t so[8], sn[8], bo[8], bn[8], bs[2][8];
  cplx coef[2];
  for (size_t j = 0; j < F->K; ++j) {
    memcpy(so, SIG(F, j), W * 8);
    if (!(parity_and(so, m1, W) & parity_and(so, m2, W))) continue;
    for (int w = 0; w < W; ++w) sn[w] = so[w] ^ f[w];
    bstar(&B, so, bo);
    bstar(&B, sn, bn);
    int m = gate_row(op, a, 0, bn, W, bs, coef);
    cplx om = {0, 0};
    for (int r = 0; r < m; ++r) {
      cplx u;
      if (amp_at(&F->t, &B, so, bo, bs[r], &u)) om = cadd(om, cmul(coef[r], u));
    }
    double mag = sqrt(om.re * om.re + om.im * om.im);
    if (fabs(mag - 1.0) > 1e-9) { fprintf(stderr, "oracle: |omega| = %g\n", mag); abort(); }
    F->amp[j] = cmul(F->amp[j], om);
    memcpy(SIG(F, j), sn, W * 8);
  }
  frame_merge(F);
  bmap_free(&B);
}

/* Direct controlled phase (Eq. 3): cofactor on c, then on t, then the phase
 * exp(i theta) on the elements where both read 1.  theta a multiple of pi is
 * Clifford (identity or CZ). */
static int frame_cphase_direct(frame_t *F, int c, int t, int64_t num, int64_t den) {
  if (den < 0) { num = -num; den = -den; }
  if (num % den == 0) {
    if ((((num / den) % 2) + 2) % 2) frame_clifford(F, OP_CZ, c, t);
    return 0;
  }
  const cplx one = {1.0, 0.0};
  frame_cofactor(F, c, one, 0);
  frame_cofactor(F, t, one, 0);
  uint64_t rc[8], rt[8];
  if (!zq_rows(&F->t, c, rc) || !zq_rows(&F->t, t, rt)) abort();
  double th = M_PI * (double)num / (double)den;
  cplx ph = {cos(th), sin(th)};
  for (size_t j = 0; j < F->K; ++j)
    if (parity_and(SIG(F, j), rc, F->W) & parity_and(SIG(F, j), rt, F->W)) F->amp[j] = cmul(F->amp[j], ph);
  return 0;
}

/* Direct Toffoli (Eq. 2): cofactor on both controls, then X on the target of
 * the elements where both controls read 1. */
static int frame_toffoli_direct(frame_t *F, int c1, int c2, int t) {
  const cplx one = {1.0, 0.0};
  frame_cofactor(F, c1, one, 0);
  frame_cofactor(F, c2, one, 0);
  uint64_t r1[8], r2[8];
  if (!zq_rows(&F->t, c1, r1) || !zq_rows(&F->t, c2, r2)) abort();
  frame_pauli_masked(F, OP_X, t, r1, r2);
  return 0;
}

/* Pairwise sum over canonical order, padded with +0.0 to a power of two. */
static double tree_sum(double *v, size_t K) {
  size_t P = 1;
  while (P < K) P <<= 1;
  double *w = calloc(P ? P : 1, sizeof(double));
  memcpy(w, v, K * sizeof(double));
  for (size_t h = P; h > 1; h >>= 1)
    for (size_t i = 0; i < h / 2; ++i) w[i] = w[2 * i] + w[2 * i + 1];
  double r = P ? w[0] : 0.0;
  free(w);
  return r;
}

static uint64_t sm64(uint64_t state, uint64_t index) {
  uint64_t z = state + (index + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Measuring F (section 4): cofactor on q, then p(1) over the merged frame,
 * a seeded biased coin, keep the consistent elements and renormalise. */
static int frame_measure(frame_t *F, int q) {
  int W = F->W;
  cplx one = {1, 0};
  frame_cofactor(F, q, one, 0);
  uint64_t rq[8];
  if (!zq_rows(&F->t, q, rq)) abort();
  double *v1 = malloc(sizeof(double) * (F->K ? F->K : 1));
  double *v0 = malloc(sizeof(double) * (F->K ? F->K : 1));
  for (size_t j = 0; j < F->K; ++j) {
    int x = parity_and(SIG(F, j), rq, W);
    volatile double rr = F->amp[j].re * F->amp[j].re;
    volatile double ii = F->amp[j].im * F->amp[j].im;
    double m2 = rr + ii;
    v1[j] = x ? m2 : 0.0;
    v0[j] = x ? 0.0 : m2;
  }
  double p1 = tree_sum(v1, F->K), p0 = tree_sum(v0, F->K);
  free(v1); free(v0);
  double u = (double)(sm64(F->seed, F->nmeas) >> 11) * (1.0 / 9007199254740992.0);
  F->nmeas++;
  if (fabs(u - p1) < FRAGILE_COIN) F->fragile = 1;
  int outcome = u < p1;
  double s = 1.0 / sqrt(outcome ? p1 : p0);
  size_t o = 0;
  for (size_t j = 0; j < F->K; ++j) {
    if (parity_and(SIG(F, j), rq, W) != outcome) continue;
    memmove(SIG(F, o), SIG(F, j), W * 8);
    F->amp[o] = cscale(F->amp[j], s);
    ++o;
  }
  F->K = o;
  if (F->nout == F->outcap) { F->outcap = F->outcap ? 2 * F->outcap : 16; F->out = realloc(F->out, F->outcap); }
  F->out[F->nout++] = (uint8_t)outcome;
  return outcome;
}

/* ------------------------------------------------------------------------- */
/* Exported C API (loaded by the Python wrapper in oracle/frame.py)           */
/* ------------------------------------------------------------------------- */
frame_t *ofr_new(int n, const uint8_t *init_bits, uint64_t seed) {
  if (n < 1 || n > 512) return NULL;
  frame_t *F = calloc(1, sizeof(frame_t));
  tab_init(&F->t, n);
  F->n = n; F->W = F->t.W; F->seed = seed;
  for (int q = 0; q < n; ++q) setbit(RZ(&F->t, q), q, 1); /* basis form: row q = Z_q (Figure 2a) */
  frame_reserve(F, 1);
  memset(F->sig, 0, F->W * 8);
  for (int q = 0; q < n; ++q) if (init_bits && init_bits[q]) setbit(F->sig, q, 1);
  F->amp[0].re = 1; F->amp[0].im = 0;
  F->K = 1;
  return F;
}

void ofr_free(frame_t *F) {
  if (!F) return;
  tab_free(&F->t); free(F->sig); free(F->amp); free(F->out); free(F);
}

static int is_clifford_angle(int64_t num, int64_t den, int *which) {
  /* theta = pi num/den is a multiple of pi/2 iff 2 num / den is an integer */
  if ((2 * num) % den != 0) return 0;
  int64_t m = (2 * num) / den;
  *which = (int)(((m % 4) + 4) % 4);
  return 1;
}

static int apply_phase_gate(frame_t *F, int q, int64_t num, int64_t den) {
  if (den < 0) { num = -num; den = -den; }
  int which;
  if (is_clifford_angle(num, den, &which)) {
    if (which == 1) frame_clifford(F, OP_S, q, 0);
    else if (which == 2) frame_clifford(F, OP_Z, q, 0);
    else if (which == 3) frame_clifford(F, OP_SDG, q, 0);
    return 0;
  }
  double th = M_PI * (double)num / (double)den;
  cplx ph = {cos(th), sin(th)};
  frame_cofactor(F, q, ph, 1);
  return 0;
}

/* Apply one gate; returns the measurement outcome for MEASURE, else 0;
 * -1 on an invalid gate. */
int ofr_apply(frame_t *F, int op, int q0, int q1, int q2, int64_t num, int64_t den) {
  int n = F->n;
  if (q0 < 0 || q0 >= n) return -1;
  switch (op) {
    case OP_H: case OP_S: case OP_SDG: case OP_X: case OP_Y: case OP_Z:
      frame_clifford(F, op, q0, 0); return 0;
    case OP_CNOT: case OP_CZ:
      if (q1 < 0 || q1 >= n || q1 == q0) return -1;
      frame_clifford(F, op, q0, q1); return 0;
    case OP_T: return apply_phase_gate(F, q0, 1, 4);
    case OP_TDG: return apply_phase_gate(F, q0, -1, 4);
    case OP_PHASE: if (den == 0) return -1; return apply_phase_gate(F, q0, num, den);
    case OP_CPHASE:
      if (den == 0 || q1 < 0 || q1 >= n || q1 == q0) return -1;
      /* phi c t = phi/2 (c + t - (c xor t)) */
      apply_phase_gate(F, q1, num, 2 * den);
      frame_clifford(F, OP_CNOT, q0, q1);
      apply_phase_gate(F, q1, -num, 2 * den);
      frame_clifford(F, OP_CNOT, q0, q1);
      apply_phase_gate(F, q0, num, 2 * den);
      return 0;
    case OP_TOF:
      if (q1 < 0 || q1 >= n || q2 < 0 || q2 >= n || q1 == q0 || q2 == q0 || q2 == q1) return -1;
      {
        /* textbook Clifford+T network: 2 H, 6 CNOT, 7 T/T-dagger */
        int c1 = q0, c2 = q1, t = q2;
        frame_clifford(F, OP_H, t, 0);
        frame_clifford(F, OP_CNOT, c2, t); apply_phase_gate(F, t, -1, 4);
        frame_clifford(F, OP_CNOT, c1, t); apply_phase_gate(F, t, 1, 4);
        frame_clifford(F, OP_CNOT, c2, t); apply_phase_gate(F, t, -1, 4);
        frame_clifford(F, OP_CNOT, c1, t); apply_phase_gate(F, c2, 1, 4); apply_phase_gate(F, t, 1, 4);
        frame_clifford(F, OP_H, t, 0);
        frame_clifford(F, OP_CNOT, c1, c2); apply_phase_gate(F, c1, 1, 4); apply_phase_gate(F, c2, -1, 4);
        frame_clifford(F, OP_CNOT, c1, c2);
      }
      return 0;
    case OP_MEASURE: return frame_measure(F, q0);
    case OP_CPHASE_D:
      if (den == 0 || q1 < 0 || q1 >= n || q1 == q0) return -1;
      return frame_cphase_direct(F, q0, q1, num, den);
    case OP_TOF_D:
      if (q1 < 0 || q1 >= n || q2 < 0 || q2 >= n || q1 == q0 || q2 == q0 || q2 == q1) return -1;
      return frame_toffoli_direct(F, q0, q1, q2);
  }
  return -1;
}

size_t ofr_size(frame_t *F) { return F->K; }
int ofr_xblock(frame_t *F) { return xblock(&F->t); }
int ofr_fragile(frame_t *F) { return F->fragile; }
size_t ofr_outcomes(frame_t *F, uint8_t *out, size_t cap) {
  size_t m = F->nout < cap ? F->nout : cap;
  if (out && m) memcpy(out, F->out, m);
  return F->nout;
}

/* tableau: n rows of [x words | z words]; sigma: K x W; amp: 2K doubles. */
size_t ofr_read(frame_t *F, uint64_t *tableau, uint64_t *sigma, double *amp, size_t cap) {
  int W = F->W;
  if (tableau)
    for (int i = 0; i < F->n; ++i) {
      memcpy(tableau + (size_t)i * 2 * W, RX(&F->t, i), W * 8);
      memcpy(tableau + (size_t)i * 2 * W + W, RZ(&F->t, i), W * 8);
    }
  if (cap >= F->K) {
    if (sigma) memcpy(sigma, F->sig, F->K * W * 8);
    if (amp) for (size_t j = 0; j < F->K; ++j) { amp[2 * j] = F->amp[j].re; amp[2 * j + 1] = F->amp[j].im; }
  }
  return F->K;
}

/* Run a whole gate list; sizes[g] receives |F| just before gate g. */
int ofr_run(frame_t *F, const int32_t *ops, const int32_t *q, const int64_t *num,
            const int64_t *den, size_t ngates, uint64_t *sizes) {
  for (size_t g = 0; g < ngates; ++g) {
    if (sizes) sizes[g] = F->K;
    if (ofr_apply(F, ops[g], q[3 * g], q[3 * g + 1], q[3 * g + 2], num[g], den[g]) < 0) return -1;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Hooks that expose single steps to the pinning tests.                       */
/* ------------------------------------------------------------------------- */
int ofr_pauli_g(int x1, int z1, int x2, int z2) { return pauli_g(x1, z1, x2, z2); }

/* Conjugate one row (bits on qubits 0..n-1, n <= 64) by a Clifford gate;
 * returns the sign flip and updates x, z in place. */
int ofr_conjugate_row(int n, int op, int a, int b, uint64_t *x, uint64_t *z) {
  tab_t t; tab_init(&t, n > 1 ? n : 1);
  t.n = 1;
  RX(&t, 0)[0] = *x; RZ(&t, 0)[0] = *z;
  uint64_t f[8];
  clifford_columns(&t, op, a, b, f);
  *x = RX(&t, 0)[0]; *z = RZ(&t, 0)[0];
  t.n = n;
  tab_free(&t);
  return (int)(f[0] & 1u);
}

/* Canonicalise an arbitrary signed generator list (n <= 64): rows[i] = (x, z),
 * sig bit i = sign of row i.  Outputs the canonical rows and signs. */
void ofr_canonicalize_signed(int n, uint64_t *x, uint64_t *z, uint64_t *sig) {
  tab_t t; tab_init(&t, n);
  for (int i = 0; i < n; ++i) { RX(&t, i)[0] = x[i]; RZ(&t, i)[0] = z[i]; }
  oplog L = {0};
  canonicalize(&t, &L);
  replay(&L, sig);
  for (int i = 0; i < n; ++i) { x[i] = RX(&t, i)[0]; z[i] = RZ(&t, i)[0]; }
  free(L.op);
  tab_free(&t);
}
