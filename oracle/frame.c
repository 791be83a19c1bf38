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

/* largest register: OW words of 64 qubits (fixed-size scratch vectors) */
#define OW 32
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
  uint64_t v[OW];
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
static int gate_row(int op, int a, int c2, const uint64_t *bp, int W, uint64_t bs[2][OW], cplx coef[2]) {
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
  uint64_t f[OW];
  clifford_columns(&F->t, op, a, b, f);
  oplog L = {0};
  canonicalize(&F->t, &L);
  bmap_t Bn; bmap_build(&Bn, &F->t);
  double scale = ldexp(1.0, 0);
  int dk = Bn.k - Bo.k; /* 2^{(k'-k)/2} */
  if (dk == 1) scale = sqrt(2.0); else if (dk == -1) scale = sqrt(0.5); else if (dk != 0) abort();
  uint64_t so[OW], sn[OW], bo[OW], bn[OW], bs[2][OW];
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
  uint64_t tgt[OW] = {0};
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
  uint64_t rq[OW];
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
  uint64_t so[OW], s1[OW], sc[OW], bo[OW], bn[OW];
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
  uint64_t f[OW];
  clifford_columns(&t2, op, a, 0, f);
  tab_free(&t2);
  bmap_t B; bmap_build(&B, &F->t);
  uint64_t so[OW], sn[OW], bo[OW], bn[OW], bs[2][OW];
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
  uint64_t rc[OW], rt[OW];
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
  uint64_t r1[OW], r2[OW];
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
  uint64_t rq[OW];
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
  if (n < 1 || n > 64 * OW) return NULL;
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
  uint64_t f[OW];
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

/* ------------------------------------------------------------------------- */
/* Multiframes (section 4, "Multiframe simulation" and "Orthogonality of      */
/* multiframes"): a list of frames F_1..F_s with their own stabilizer         */
/* matrices; the state is the sum of every frame's expansion.                 */
/*                                                                            */
/* Readings (the paper leaves these open):                                    */
/*  - Coalescing runs after every gate that cofactors (non-Clifford phase     */
/*    gates, the direct controlled phase and Toffoli); the 7-T Toffoli and    */
/*    the three-phase-gate controlled phase are applied gate by gate.         */
/*  - Candidate pairs: elements are scanned in canonical order; an unpaired   */
/*    element takes, among the later unpaired elements that differ from it   */
/*    only on Z_k rows (rows equal to +-Z_k) and whose amplitude equals its   */
/*    own times i^d (d in 0..3, relative tolerance COAL_TOL), the one that    */
/*    differs on the fewest rows (then the first in canonical order).         */
/*  - Orientation: v_1 is the smallest qubit of the differing Z_k rows, r'    */
/*    the element of the pair whose sign on the Z_{v_1} row is +, and d is    */
/*    fixed by a_j' = i^d a_r'.  Then a_r' psi_r' + a_j' psi_j' =             */
/*    sqrt2 a_r' C psi_r' with C = CNOT_{v1,v2}..CNOT_{v1,vm} P^d H_{v1}      */
/*    (Step 3 of COALESCE), so the coalesced element is the element           */
/*    (sigma_r', sqrt2 a_r') rotated by C; every pair of one class (same      */
/*    differing rows, same d) goes to one new frame with matrix C M C^dag.    */
/*  - Frames are kept sorted by their canonical matrix (row-major words);     */
/*    frames with equal matrices are merged (equal phase vectors add).        */
/*  - Measurement: cofactor every frame on q, merge equal matrices, check     */
/*    Invariant 2 exactly and orthogonalize if it fails, then p(1) as the     */
/*    pairwise tree sum over the frames in order and their elements in       */
/*    canonical order, the coin, and the filter.                              */
/*  - Orthogonality of two states: psi_A and psi_B are orthogonal exactly     */
/*    when some Pauli P has P in S(psi_A) and -P in S(psi_B) (the footnote of */
/*    Observation 2; the converse holds for stabilizer states).  P ranges    */
/*    over the intersection of the two unsigned groups; the sign difference  */
/*    is linear on it, so a basis of the intersection decides.               */
/*  - Orthogonalization pivot: the smallest qubit whose column carries a      */
/*    different set of Pauli literals in two of the frames' matrices; if no   */
/*    column does but several frames remain, the smallest qubit whose column  */
/*    differs at all.                                                         */
/* ------------------------------------------------------------------------- */
#define COAL_TOL 1e-9

typedef struct {
  int n, W;
  frame_t **fr;
  size_t nf, cap;
  uint64_t seed, nmeas;
  uint8_t *out;
  size_t nout, outcap;
  int fragile;
  int general;  /* coalesce through the basis circuit (the extension) */
  size_t ortho_runs, coalesced;
} mframe_t;

static frame_t *frame_empty_like(const frame_t *src) {
  frame_t *F = calloc(1, sizeof(frame_t));
  tab_copy(&F->t, &src->t);
  F->n = src->n; F->W = src->W;
  frame_reserve(F, 1);
  F->K = 0;
  return F;
}

static void frame_push(frame_t *F, const uint64_t *sig, cplx a) {
  frame_reserve(F, F->K + 1);
  memcpy(SIG(F, F->K), sig, F->W * 8);
  F->amp[F->K] = a;
  F->K++;
}

static void frame_destroy(frame_t *F) { ofr_free(F); }

static int tab_cmp(const tab_t *a, const tab_t *b) {
  size_t words = (size_t)a->n * a->W;
  for (size_t i = 0; i < (size_t)a->n; ++i) {
    int c = memcmp(a->x + i * a->W, b->x + i * a->W, a->W * 8);
    if (c) return c;
    c = memcmp(a->z + i * a->W, b->z + i * a->W, a->W * 8);
    if (c) return c;
  }
  (void)words;
  return 0;
}

static void mf_push(mframe_t *M, frame_t *F) {
  if (M->nf == M->cap) { M->cap = M->cap ? 2 * M->cap : 8; M->fr = realloc(M->fr, M->cap * sizeof(frame_t *)); }
  M->fr[M->nf++] = F;
}

static int frame_ptr_cmp(const void *a, const void *b) {
  const frame_t *x = *(frame_t *const *)a, *y = *(frame_t *const *)b;
  return tab_cmp(&x->t, &y->t);
}

/* Merge frames with equal matrices, drop empty frames, sort by matrix. */
static void mf_merge_equal(mframe_t *M) {
  qsort(M->fr, M->nf, sizeof(frame_t *), frame_ptr_cmp);
  size_t o = 0;
  for (size_t i = 0; i < M->nf;) {
    frame_t *F = M->fr[i];
    size_t j = i + 1;
    int grew = 0;
    while (j < M->nf && tab_cmp(&M->fr[j]->t, &F->t) == 0) {
      frame_t *G = M->fr[j];
      for (size_t e = 0; e < G->K; ++e) frame_push(F, SIG(G, e), G->amp[e]);
      frame_destroy(G);
      grew = 1;
      ++j;
    }
    if (grew) frame_merge(F);
    if (F->fragile) M->fragile = 1;
    if (F->K) M->fr[o++] = F;
    else frame_destroy(F);
    i = j;
  }
  M->nf = o;
}

/* COALESCE(F) (section 4): candidate pairs leave F and become the elements of
 * new frames appended to M.  Returns the number of pairs coalesced. */
static size_t frame_coalesce(frame_t *F, mframe_t *M) {
  const int n = F->n, W = F->W;
  uint64_t zr[OW] = {0};
  int *zq = malloc(sizeof(int) * (size_t)n);
  for (int i = 0; i < n; ++i) {
    int xany = 0, zc = 0;
    for (int w = 0; w < W; ++w) { xany |= RX(&F->t, i)[w] != 0; zc += __builtin_popcountll(RZ(&F->t, i)[w]); }
    zq[i] = (!xany && zc == 1) ? lowest_bit(RZ(&F->t, i), W) : -1;
    if (zq[i] >= 0) setbit(zr, i, 1);
  }
  const size_t K = F->K;
  long *part = malloc(sizeof(long) * (K ? K : 1));
  int *dd = malloc(sizeof(int) * (K ? K : 1));
  for (size_t j = 0; j < K; ++j) part[j] = -1;
  size_t npairs = 0;
  uint64_t diff[OW];
  for (size_t r = 0; r < K; ++r) {
    if (part[r] >= 0) continue;
    long best = -1;
    int bestpop = 1 << 30, bestd = 0;
    for (size_t j = r + 1; j < K; ++j) {
      if (part[j] >= 0) continue;
      int outside = 0, pop = 0, e1 = -1, v1 = 1 << 30;
      for (int w = 0; w < W; ++w) {
        diff[w] = SIG(F, r)[w] ^ SIG(F, j)[w];
        outside |= (diff[w] & ~zr[w]) != 0;
        pop += __builtin_popcountll(diff[w]);
      }
      if (outside || pop == 0 || pop >= bestpop) continue;
      for (int i = 0; i < n; ++i)
        if (getbit(diff, i) && zq[i] < v1) { v1 = zq[i]; e1 = i; }
      /* r' has sign + on the Z_{v1} row */
      size_t rp = getbit(SIG(F, r), e1) ? j : r, jp = rp == r ? j : r;
      cplx ar = F->amp[rp], aj = F->amp[jp];
      double mr = sqrt(ar.re * ar.re + ar.im * ar.im), mj = sqrt(aj.re * aj.re + aj.im * aj.im);
      double tol = COAL_TOL * (mr > mj ? mr : mj);
      for (int d = 0; d < 4; ++d) {
        cplx t = cmul(ipow(d), ar);
        if (fabs(aj.re - t.re) <= tol && fabs(aj.im - t.im) <= tol) {
          best = (long)j; bestpop = pop; bestd = d;
          break;
        }
      }
    }
    if (best >= 0) {
      part[r] = best; part[best] = (long)r;
      dd[r] = dd[best] = bestd;
      ++npairs;
    }
  }
  if (npairs) {
    /* classes in order of their first pair (canonical order of r) */
    uint8_t *done = calloc(K ? K : 1, 1);
    for (size_t r = 0; r < K; ++r) {
      if (part[r] < 0 || done[r] || (size_t)part[r] < r) continue;
      uint64_t cls[OW];
      for (int w = 0; w < W; ++w) cls[w] = SIG(F, r)[w] ^ SIG(F, part[r])[w];
      const int dcls = dd[r];
      int v[64 * OW] = {0}, m = 0;
      for (int i = 0; i < n; ++i) if (getbit(cls, i)) v[m++] = zq[i];
      /* v ascending */
      for (int a = 0; a < m; ++a)
        for (int b = a + 1; b < m; ++b)
          if (v[b] < v[a]) { int t = v[a]; v[a] = v[b]; v[b] = t; }
      int e1 = -1;
      for (int i = 0; i < n; ++i) if (getbit(cls, i) && zq[i] == v[0]) e1 = i;
      frame_t *N = frame_empty_like(F);
      for (size_t s = r; s < K; ++s) {
        if (part[s] < 0 || done[s] || (size_t)part[s] < s || dd[s] != dcls) continue;
        int same = 1;
        for (int w = 0; w < W; ++w) same &= (SIG(F, s)[w] ^ SIG(F, part[s])[w]) == cls[w];
        if (!same) continue;
        size_t rp = getbit(SIG(F, s), e1) ? (size_t)part[s] : s;
        frame_push(N, SIG(F, rp), cscale(F->amp[rp], sqrt(2.0)));
        done[s] = done[part[s]] = 1;
      }
      frame_sort(N);
      frame_clifford(N, OP_H, v[0], 0);
      if (dcls == 1) frame_clifford(N, OP_S, v[0], 0);
      else if (dcls == 2) frame_clifford(N, OP_Z, v[0], 0);
      else if (dcls == 3) frame_clifford(N, OP_SDG, v[0], 0);
      for (int l = 1; l < m; ++l) frame_clifford(N, OP_CNOT, v[0], v[l]);
      if (N->fragile) M->fragile = 1;
      mf_push(M, N);
    }
    free(done);
    /* the unpaired elements stay */
    size_t o = 0;
    for (size_t j = 0; j < K; ++j) {
      if (part[j] >= 0) continue;
      memmove(SIG(F, o), SIG(F, j), W * 8);
      F->amp[o] = F->amp[j];
      ++o;
    }
    F->K = o;
  }
  free(part); free(dd); free(zq);
  return npairs;
}

/* A stabilizer circuit C (gate list, applied in order) with C G C^dag =
 * <Z_0, .., Z_{n-1}> for the unsigned group G of a canonical matrix
 * (Corollary: every stabilizer matrix maps to the basis form of Figure 2a):
 * CNOTs make every X-block row's x part its pivot alone, S and CZ clear its
 * z part, H turns it into Z at the pivot, and CNOTs reduce the Z-type rows
 * to single Z's.  Returns the number of gates (3 ints each: op, a, b). */
static int basis_circuit(const tab_t *src, int *gates) {
  tab_t t; tab_copy(&t, src);
  int n = t.n, W = t.W, ng = 0, k = xblock(&t);
  uint64_t f[OW];
#define EMIT(o, a, b) do { gates[3 * ng] = (o); gates[3 * ng + 1] = (a); gates[3 * ng + 2] = (b); ++ng; \
                           clifford_columns(&t, (o), (a), (b), f); } while (0)
  int *piv = malloc(sizeof(int) * (n ? n : 1));
  for (int l = 0; l < k; ++l) piv[l] = lowest_bit(RX(&t, l), W);
  for (int l = 0; l < k; ++l)
    for (int j = 0; j < n; ++j)
      if (j != piv[l] && getbit(RX(&t, l), j)) EMIT(OP_CNOT, piv[l], j);
  for (int l = 0; l < k; ++l) {
    if (getbit(RZ(&t, l), piv[l])) EMIT(OP_S, piv[l], 0);
    for (int j = 0; j < n; ++j)
      if (j != piv[l] && getbit(RZ(&t, l), j)) EMIT(OP_CZ, piv[l], j);
  }
  for (int l = 0; l < k; ++l) EMIT(OP_H, piv[l], 0);
  /* now every row is Z-type: reduce, then clear each row off its pivot */
  oplog L = {0};
  canonicalize(&t, &L);
  free(L.op);
  for (int i = 0; i < n; ++i) {
    int q = lowest_bit(RZ(&t, i), W);
    for (int j = 0; j < n; ++j)
      if (j != q && getbit(RZ(&t, i), j)) EMIT(OP_CNOT, j, q);
  }
#undef EMIT
  for (int i = 0; i < n; ++i) {
    int bad = 0;
    for (int w = 0; w < W; ++w) bad |= RX(&t, i)[w] != 0;
    if (bad || __builtin_popcountll(RZ(&t, i)[lowest_bit(RZ(&t, i), W) >> 6]) != 1) {
      fprintf(stderr, "oracle: basis circuit left a row that is not a single Z\n");
      abort();
    }
  }
  free(piv);
  tab_free(&t);
  return ng;
}

static void frame_rotate(frame_t *F, const int *gates, int ng, int inverse) {
  if (!inverse) {
    for (int g = 0; g < ng; ++g) frame_clifford(F, gates[3 * g], gates[3 * g + 1], gates[3 * g + 2]);
  } else {
    for (int g = ng - 1; g >= 0; --g) {
      int op = gates[3 * g];
      if (op == OP_S) op = OP_SDG;
      else if (op == OP_SDG) op = OP_S;
      frame_clifford(F, op, gates[3 * g + 1], gates[3 * g + 2]);
    }
  }
}

/* The extension of COALESCE to matrices without Z_k rows (section 4): find
 * C mapping M to the basis form, ROTATE(F, C), COALESCE, and ROTATE every
 * resulting frame by C^dag. */
static size_t frame_coalesce_general(frame_t *F, mframe_t *M) {
  const int n = F->n;
  int *gates = malloc(sizeof(int) * 3 * (size_t)(4 * n * n + 4 * n + 8));
  int ng = basis_circuit(&F->t, gates);
  frame_rotate(F, gates, ng, 0);
  mframe_t tmp = {0};
  tmp.n = M->n; tmp.W = M->W;
  size_t made = frame_coalesce(F, &tmp);
  frame_rotate(F, gates, ng, 1);
  for (size_t i = 0; i < tmp.nf; ++i) {
    frame_rotate(tmp.fr[i], gates, ng, 1);
    if (tmp.fr[i]->fragile) M->fragile = 1;
    mf_push(M, tmp.fr[i]);
  }
  if (F->fragile) M->fragile = 1;
  free(tmp.fr);
  free(gates);
  return made;
}

static void mf_coalesce_all(mframe_t *M) {
  for (;;) {
    size_t made = 0, nf0 = M->nf;
    for (size_t i = 0; i < nf0; ++i)
      made += M->general ? frame_coalesce_general(M->fr[i], M) : frame_coalesce(M->fr[i], M);
    mf_merge_equal(M);
    M->coalesced += made;
    if (!made) break;
  }
}

/* Sign of the product of the rows of `t` selected by mask c, as
 * sign(prod_i in c (-1)^{sig_i} row_i) = sig.c ^ kappa(c): kappa from the
 * Pauli products (Table 1) of the unsigned rows, applied left to right. */
static int product_kappa(tab_t *t, const uint64_t *c, uint64_t *px, uint64_t *pz) {
  int W = t->W, e = 0;
  memset(px, 0, W * 8); memset(pz, 0, W * 8);
  for (int i = 0; i < t->n; ++i) {
    if (!getbit(c, i)) continue;
    for (int q = 0; q < t->n; ++q)
      e += pauli_g(getbit(px, q), getbit(pz, q), getbit(RX(t, i), q), getbit(RZ(t, i), q));
    for (int w = 0; w < W; ++w) { px[w] ^= RX(t, i)[w]; pz[w] ^= RZ(t, i)[w]; }
  }
  e = ((e % 4) + 4) % 4;
  if (e & 1) { fprintf(stderr, "oracle: non-Hermitian product\n"); abort(); }
  return e >> 1;
}

/* Basis of the intersection of the unsigned groups of two canonical
 * matrices: for each basis element t, the row masks cA[t], cB[t] and the
 * constants kA[t], kB[t].  Returns the number of basis elements. */
static int intersection(tab_t *A, tab_t *B, uint64_t *cA, uint64_t *cB, int *kA, int *kB) {
  int n = A->n, W = A->W;
  /* pivots of A (fully reduced: row i's pivot column) */
  int *pa = malloc(sizeof(int) * n);
  for (int i = 0; i < n; ++i) {
    pa[i] = -1;
    for (int col = 0; col < 2 * n && pa[i] < 0; ++col) if (colbit(A, i, col)) pa[i] = col;
  }
  /* residuals of B's rows against A, with the combination tracked */
  uint64_t *rx = calloc((size_t)n * W, 8), *rz = calloc((size_t)n * W, 8), *cb = calloc((size_t)n * W, 8);
  for (int j = 0; j < n; ++j) {
    memcpy(rx + (size_t)j * W, RX(B, j), W * 8);
    memcpy(rz + (size_t)j * W, RZ(B, j), W * 8);
    for (int i = 0; i < n; ++i) {
      int col = pa[i];
      int bit = col < n ? getbit(rx + (size_t)j * W, col) : getbit(rz + (size_t)j * W, col - n);
      if (bit)
        for (int w = 0; w < W; ++w) { rx[(size_t)j * W + w] ^= RX(A, i)[w]; rz[(size_t)j * W + w] ^= RZ(A, i)[w]; }
    }
    setbit(cb + (size_t)j * W, j, 1);
  }
  /* null space of the residuals: eliminate, tracking combinations */
  int r = 0;
  for (int col = 0; col < 2 * n; ++col) {
    int p = -1;
    for (int j = r; j < n; ++j) {
      int bit = col < n ? getbit(rx + (size_t)j * W, col) : getbit(rz + (size_t)j * W, col - n);
      if (bit) { p = j; break; }
    }
    if (p < 0) continue;
    for (int w = 0; w < W; ++w) {
      uint64_t t;
      t = rx[(size_t)p * W + w]; rx[(size_t)p * W + w] = rx[(size_t)r * W + w]; rx[(size_t)r * W + w] = t;
      t = rz[(size_t)p * W + w]; rz[(size_t)p * W + w] = rz[(size_t)r * W + w]; rz[(size_t)r * W + w] = t;
      t = cb[(size_t)p * W + w]; cb[(size_t)p * W + w] = cb[(size_t)r * W + w]; cb[(size_t)r * W + w] = t;
    }
    for (int j = 0; j < n; ++j) {
      if (j == r) continue;
      int bit = col < n ? getbit(rx + (size_t)j * W, col) : getbit(rz + (size_t)j * W, col - n);
      if (bit)
        for (int w = 0; w < W; ++w) {
          rx[(size_t)j * W + w] ^= rx[(size_t)r * W + w];
          rz[(size_t)j * W + w] ^= rz[(size_t)r * W + w];
          cb[(size_t)j * W + w] ^= cb[(size_t)r * W + w];
        }
    }
    ++r;
  }
  int nb = 0;
  uint64_t gx[OW], gz[OW];
  for (int j = r; j < n; ++j) {
    /* combination cb[j] of B's rows lies in span(A) */
    memcpy(cB + (size_t)nb * W, cb + (size_t)j * W, W * 8);
    kB[nb] = product_kappa(B, cB + (size_t)nb * W, gx, gz);
    memset(cA + (size_t)nb * W, 0, W * 8);
    for (int i = 0; i < n; ++i) {
      int col = pa[i];
      if (col < n ? getbit(gx, col) : getbit(gz, col - n)) setbit(cA + (size_t)nb * W, i, 1);
    }
    uint64_t hx[OW], hz[OW];
    kA[nb] = product_kappa(A, cA + (size_t)nb * W, hx, hz);
    for (int w = 0; w < W; ++w)
      if (hx[w] != gx[w] || hz[w] != gz[w]) { fprintf(stderr, "oracle: intersection element outside span\n"); abort(); }
    ++nb;
  }
  free(pa); free(rx); free(rz); free(cb);
  return nb;
}

/* Invariant 2 between two frames: every state of A is orthogonal to every
 * state of B (frames with distinct matrices). */
static int frames_orthogonal(frame_t *A, frame_t *B) {
  int n = A->n, W = A->W;
  uint64_t *cA = calloc((size_t)n * W, 8), *cB = calloc((size_t)n * W, 8);
  int *kA = malloc(sizeof(int) * n), *kB = malloc(sizeof(int) * n);
  int nb = intersection(&A->t, &B->t, cA, cB, kA, kB);
  int ok = 1;
  for (size_t i = 0; i < A->K && ok; ++i)
    for (size_t j = 0; j < B->K && ok; ++j) {
      int differ = 0;
      for (int t = 0; t < nb && !differ; ++t)
        differ = (parity_and(SIG(A, i), cA + (size_t)t * W, W) ^ kA[t]) !=
                 (parity_and(SIG(B, j), cB + (size_t)t * W, W) ^ kB[t]);
      if (!differ) ok = 0;
    }
  free(cA); free(cB); free(kA); free(kB);
  return ok;
}

static int mf_orthogonal(mframe_t *M) {
  for (size_t a = 0; a < M->nf; ++a)
    for (size_t b = a + 1; b < M->nf; ++b)
      if (!frames_orthogonal(M->fr[a], M->fr[b])) return 0;
  return 1;
}

/* literal set of column q of a matrix: bit 0 I, 1 Z, 2 X, 3 Y present */
static int literal_set(tab_t *t, int q) {
  int s = 0;
  for (int i = 0; i < t->n; ++i) s |= 1 << (2 * getbit(RX(t, i), q) + getbit(RZ(t, i), q));
  return s;
}

static int column_differs(tab_t *a, tab_t *b, int q) {
  for (int i = 0; i < a->n; ++i)
    if (getbit(RX(a, i), q) != getbit(RX(b, i), q) || getbit(RZ(a, i), q) != getbit(RZ(b, i), q)) return 1;
  return 0;
}

/* Orthogonalization (section 4): cofactor every frame on a pivot qubit and
 * merge frames with equal matrices until one frame remains. */
static void mf_orthogonalize(mframe_t *M) {
  const cplx one = {1.0, 0.0};
  M->ortho_runs++;
  while (M->nf > 1) {
    int p = -1;
    for (int q = 0; q < M->n && p < 0; ++q) {
      int s0 = literal_set(&M->fr[0]->t, q);
      for (size_t i = 1; i < M->nf && p < 0; ++i) if (literal_set(&M->fr[i]->t, q) != s0) p = q;
    }
    for (int q = 0; q < M->n && p < 0; ++q)
      for (size_t i = 1; i < M->nf && p < 0; ++i) if (column_differs(&M->fr[0]->t, &M->fr[i]->t, q)) p = q;
    if (p < 0) break; /* equal matrices: merged below */
    for (size_t i = 0; i < M->nf; ++i) frame_cofactor(M->fr[i], p, one, 0);
    mf_merge_equal(M);
  }
  mf_merge_equal(M);
}

static int mf_measure(mframe_t *M, int q) {
  const cplx one = {1.0, 0.0};
  int W = M->W;
  for (size_t i = 0; i < M->nf; ++i) frame_cofactor(M->fr[i], q, one, 0);
  mf_merge_equal(M);
  if (!mf_orthogonal(M)) mf_orthogonalize(M);
  size_t tot = 0;
  for (size_t i = 0; i < M->nf; ++i) tot += M->fr[i]->K;
  double *v1 = malloc(sizeof(double) * (tot ? tot : 1)), *v0 = malloc(sizeof(double) * (tot ? tot : 1));
  uint64_t rq[OW];
  size_t k = 0;
  for (size_t i = 0; i < M->nf; ++i) {
    frame_t *F = M->fr[i];
    if (!zq_rows(&F->t, q, rq)) abort();
    for (size_t j = 0; j < F->K; ++j, ++k) {
      int x = parity_and(SIG(F, j), rq, W);
      volatile double rr = F->amp[j].re * F->amp[j].re;
      volatile double ii = F->amp[j].im * F->amp[j].im;
      double m2 = rr + ii;
      v1[k] = x ? m2 : 0.0;
      v0[k] = x ? 0.0 : m2;
    }
  }
  double p1 = tree_sum(v1, tot), p0 = tree_sum(v0, tot);
  free(v1); free(v0);
  double u = (double)(sm64(M->seed, M->nmeas) >> 11) * (1.0 / 9007199254740992.0);
  M->nmeas++;
  if (fabs(u - p1) < FRAGILE_COIN) M->fragile = 1;
  int outcome = u < p1;
  double s = 1.0 / sqrt(outcome ? p1 : p0);
  for (size_t i = 0; i < M->nf; ++i) {
    frame_t *F = M->fr[i];
    zq_rows(&F->t, q, rq);
    size_t o = 0;
    for (size_t j = 0; j < F->K; ++j) {
      if (parity_and(SIG(F, j), rq, W) != outcome) continue;
      memmove(SIG(F, o), SIG(F, j), W * 8);
      F->amp[o] = cscale(F->amp[j], s);
      ++o;
    }
    F->K = o;
  }
  mf_merge_equal(M);
  if (M->nout == M->outcap) { M->outcap = M->outcap ? 2 * M->outcap : 16; M->out = realloc(M->out, M->outcap); }
  M->out[M->nout++] = (uint8_t)outcome;
  return outcome;
}

mframe_t *omf_new(int n, const uint8_t *init_bits, uint64_t seed) {
  frame_t *F = ofr_new(n, init_bits, seed);
  if (!F) return NULL;
  mframe_t *M = calloc(1, sizeof(mframe_t));
  M->n = n; M->W = F->W; M->seed = seed;
  mf_push(M, F);
  return M;
}

void omf_free(mframe_t *M) {
  if (!M) return;
  for (size_t i = 0; i < M->nf; ++i) frame_destroy(M->fr[i]);
  free(M->fr); free(M->out); free(M);
}

static int is_cofactoring(int op, int64_t num, int64_t den) {
  int which;
  if (op == OP_T || op == OP_TDG) return 1;
  if (op == OP_PHASE) { if (den < 0) { num = -num; den = -den; } return !is_clifford_angle(num, den, &which); }
  if (op == OP_CPHASE_D) { if (den < 0) { num = -num; den = -den; } return num % den != 0; }
  return op == OP_TOF_D;
}

/* Apply one gate to a multiframe; returns the outcome of MEASURE, else 0;
 * -1 on an invalid gate. */
int omf_apply(mframe_t *M, int op, int q0, int q1, int q2, int64_t num, int64_t den) {
  int n = M->n;
  if (q0 < 0 || q0 >= n) return -1;
  if (op == OP_MEASURE) return mf_measure(M, q0);
  if (op == OP_TOF) {
    if (q1 < 0 || q1 >= n || q2 < 0 || q2 >= n || q1 == q0 || q2 == q0 || q2 == q1) return -1;
    int c1 = q0, c2 = q1, t = q2;
    omf_apply(M, OP_H, t, 0, 0, 0, 1);
    omf_apply(M, OP_CNOT, c2, t, 0, 0, 1); omf_apply(M, OP_TDG, t, 0, 0, 0, 1);
    omf_apply(M, OP_CNOT, c1, t, 0, 0, 1); omf_apply(M, OP_T, t, 0, 0, 0, 1);
    omf_apply(M, OP_CNOT, c2, t, 0, 0, 1); omf_apply(M, OP_TDG, t, 0, 0, 0, 1);
    omf_apply(M, OP_CNOT, c1, t, 0, 0, 1); omf_apply(M, OP_T, c2, 0, 0, 0, 1); omf_apply(M, OP_T, t, 0, 0, 0, 1);
    omf_apply(M, OP_H, t, 0, 0, 0, 1);
    omf_apply(M, OP_CNOT, c1, c2, 0, 0, 1); omf_apply(M, OP_T, c1, 0, 0, 0, 1); omf_apply(M, OP_TDG, c2, 0, 0, 0, 1);
    omf_apply(M, OP_CNOT, c1, c2, 0, 0, 1);
    return 0;
  }
  if (op == OP_CPHASE) {
    if (den == 0 || q1 < 0 || q1 >= n || q1 == q0) return -1;
    omf_apply(M, OP_PHASE, q1, 0, 0, num, 2 * den);
    omf_apply(M, OP_CNOT, q0, q1, 0, 0, 1);
    omf_apply(M, OP_PHASE, q1, 0, 0, -num, 2 * den);
    omf_apply(M, OP_CNOT, q0, q1, 0, 0, 1);
    omf_apply(M, OP_PHASE, q0, 0, 0, num, 2 * den);
    return 0;
  }
  for (size_t i = 0; i < M->nf; ++i)
    if (ofr_apply(M->fr[i], op, q0, q1, q2, num, den) < 0) return -1;
  for (size_t i = 0; i < M->nf; ++i) if (M->fr[i]->fragile) M->fragile = 1;
  if (is_cofactoring(op, num, den)) mf_coalesce_all(M);
  else mf_merge_equal(M);
  return 0;
}

int omf_run(mframe_t *M, const int32_t *ops, const int32_t *q, const int64_t *num, const int64_t *den,
            size_t ngates, uint64_t *sizes, uint64_t *nframes) {
  for (size_t g = 0; g < ngates; ++g) {
    size_t tot = 0;
    for (size_t i = 0; i < M->nf; ++i) tot += M->fr[i]->K;
    if (sizes) sizes[g] = tot;
    if (nframes) nframes[g] = M->nf;
    if (omf_apply(M, ops[g], q[3 * g], q[3 * g + 1], q[3 * g + 2], num[g], den[g]) < 0) return -1;
  }
  return 0;
}

size_t omf_nframes(mframe_t *M) { return M->nf; }
size_t omf_frame_size(mframe_t *M, size_t i) { return i < M->nf ? M->fr[i]->K : 0; }
size_t omf_read(mframe_t *M, size_t i, uint64_t *tableau, uint64_t *sigma, double *amp, size_t cap) {
  if (i >= M->nf) return 0;
  return ofr_read(M->fr[i], tableau, sigma, amp, cap);
}
int omf_fragile(mframe_t *M) { return M->fragile; }
int omf_orthogonal(mframe_t *M) { return mf_orthogonal(M); }
size_t omf_ortho_runs(mframe_t *M) { return M->ortho_runs; }
size_t omf_outcomes(mframe_t *M, uint8_t *out, size_t cap) {
  size_t m = M->nout < cap ? M->nout : cap;
  if (out && m) memcpy(out, M->out, m);
  return M->nout;
}

/* A multiframe of one frame given explicitly (canonical matrix, sorted
 * distinct phase vectors, amplitudes): for pinning the frame operations. */
mframe_t *omf_load(int n, const uint64_t *tableau, const uint64_t *sigma, const double *amp, size_t K,
                   uint64_t seed) {
  mframe_t *M = omf_new(n, NULL, seed);
  if (!M) return NULL;
  frame_t *F = M->fr[0];
  int W = F->W;
  for (int i = 0; i < n; ++i) {
    memcpy(RX(&F->t, i), tableau + (size_t)i * 2 * W, W * 8);
    memcpy(RZ(&F->t, i), tableau + (size_t)i * 2 * W + W, W * 8);
  }
  F->K = 0;
  for (size_t j = 0; j < K; ++j) {
    cplx a = {amp[2 * j], amp[2 * j + 1]};
    frame_push(F, sigma + j * W, a);
  }
  frame_sort(F);
  return M;
}

/* COALESCE on every frame and the merge of equal matrices, until no pair is
 * left (the step run after every cofactoring gate); returns the pairs. */
size_t omf_coalesce(mframe_t *M) {
  size_t before = M->coalesced;
  mf_coalesce_all(M);
  return M->coalesced - before;
}

/* Invariant 2 check and, if it fails, the orthogonalization. */
int omf_orthogonalize(mframe_t *M) {
  if (mf_orthogonal(M)) return 0;
  mf_orthogonalize(M);
  return 1;
}

/* Append one explicit frame (canonical matrix, distinct phase vectors,
 * amplitudes) to a multiframe; frames with equal matrices merge. */
int omf_add_frame(mframe_t *M, const uint64_t *tableau, const uint64_t *sigma, const double *amp, size_t K) {
  frame_t *F = frame_empty_like(M->fr[0]);
  int W = F->W;
  for (int i = 0; i < M->n; ++i) {
    memcpy(RX(&F->t, i), tableau + (size_t)i * 2 * W, W * 8);
    memcpy(RZ(&F->t, i), tableau + (size_t)i * 2 * W + W, W * 8);
  }
  for (size_t j = 0; j < K; ++j) {
    cplx a = {amp[2 * j], amp[2 * j + 1]};
    frame_push(F, sigma + j * W, a);
  }
  frame_sort(F);
  mf_push(M, F);
  mf_merge_equal(M);
  return 0;
}

/* Choose the basic COALESCE (0: Z_k rows of the matrix as it is) or its
 * extension through the basis circuit (1). */
void omf_set_general(mframe_t *M, int general) { M->general = general; }
