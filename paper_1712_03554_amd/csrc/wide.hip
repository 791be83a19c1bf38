// Frames of up to 2048 qubits for stabilizer circuits (H, S, S-dagger, Pauli,
// CNOT and CZ gates and Z measurements; the random-stabilizer-circuit
// experiment of section 6).  Such a frame keeps one element (Definition 1
// with |F| = 1): the matrix M, its phase vector sigma and an amplitude a.
//
// The rows do not fit one workgroup's LDS (n = 1024 takes 256 KiB), so they
// stay in device memory (L2-resident while a frame runs) and one workgroup of
// eight wavefronts works on a frame, one row per thread and pass.  Per frame
// the workgroup keeps in LDS: sigma, b* (the smallest basis string of the
// support of psi(M, sigma)), every row's lead and the masks of the repair.
//
// Form of M between gates: X-block rows (some x bit) have distinct x-leads
// (lowest x bit) and each x-lead column has an x bit in its own row only;
// Z-block rows (no x bit) have distinct z-leads and each z-lead column has a
// z bit in its own Z-block row only (the echelon form of Figure 2b without
// the row order; readout sorts and fully reduces it).  Rows are slots: slot i
// owns sigma bit i.
//
// Clifford gate U (section 3, ROTATE with global-phase maintenance): the
// columns of the gate's qubits are conjugated (Table 2) and each row's sign
// flip goes into sigma; the form is repaired by row multiplications, each
// replayed on sigma.  The factor omega with U psi(M, sigma) = omega
// psi(M', sigma') is the ratio of the two sides at one basis string s of the
// new support.  s is picked before the gate so that <s|U psi> is known from
// b* alone (a permutation gate maps |b*> to a multiple of |s>; for H, s is b*
// or b* ^ e_a and needs the old amplitude at b* ^ e_a, one X-block row).
// After the gate psi(M', sigma')(s) follows from the X-block rows whose
// x-leads are set in s: their product P applied to |b'*> gives s, so
// b'* = s ^ x(P) and the amplitude is the phase of P |b'*> (the generators
// commute, so the product can be formed in any order).  b'* is carried to the
// next gate.
//
// Measurement of qubit q (section 4, measuring F): if an X-block row has an x
// bit at q it is multiplied into every other such row and replaced by
// (-1)^x Z_q (COFACTOR); both children have |c_x|^2 = |a|^2 / 2, so the coin
// needs no second element, and the kept child's amplitude comes from the old
// amplitude at b* or at b* ^ x(row), whichever lies in the child.  Otherwise
// a Z-block row equals Z_q and its sign is the outcome.
#include <hip/hip_runtime.h>

#include "sf_dev.h"

#define SF_WIDE_NMAX 2048
#define SF_WIDE_WMAX (SF_WIDE_NMAX / 64)
#define WT 512               // threads per frame (eight wavefronts)
#define WWAVES (WT / 64)

// Per-frame header; rows and vectors follow it in the same allocation.  The
// error field sits where TrackState keeps its own, so one check serves both.
struct WideHdr {
  int32_t n, W, k, nmeas;   // k: X-block rows; nmeas: measurements done
  int32_t pad0[6];
  int32_t error;            // int slot 10
  int32_t pad1[5];
  double2 amp;              // byte 64
  uint64_t seed;
  uint64_t pad2[5];         // 128 bytes
};
static_assert(offsetof(WideHdr, error) == 10 * 4, "error slot");
static_assert(sizeof(WideHdr) == 128, "header size");

// Layout after the header (8-byte words): rx[n W], rz[n W], sig[W], bst[W],
// then lead[n] as int32.
struct WideLayout {
  size_t rx, rz, sig, bst, lead, bytes;
};
static inline __host__ __device__ WideLayout wide_layout(int n) {
  const size_t W = (size_t)(n + 63) / 64;
  WideLayout o;
  o.rx = sizeof(WideHdr);
  o.rz = o.rx + (size_t)n * W * 8;
  o.sig = o.rz + (size_t)n * W * 8;
  o.bst = o.sig + W * 8;
  o.lead = o.bst + W * 8;
  o.bytes = o.lead + (size_t)n * 4;
  return o;
}

struct WideJob {
  unsigned char* base;      // header + layout
  const DGate* gates;
  int32_t g0, g1;           // device gates [g0, g1)
  uint8_t* outcomes;        // measurement index -> outcome
  double* pvals;            // measurement index -> p(1)
  int* flags;               // bit 0: a coin fell within 1e-12 of p(1)
};

struct WideLds {
  uint64_t sig[SF_WIDE_WMAX], bst[SF_WIDE_WMAX], s[SF_WIDE_WMAX];
  // candidate columns of the repair and z bits of rows that left the X-block
  // (bit b: x column b for b < 64 W, z column b - 64 W above)
  uint64_t cand[2 * SF_WIDE_WMAX], zpend[SF_WIDE_WMAX];
  uint64_t px[WWAVES][SF_WIDE_WMAX], pz[WWAVES][SF_WIDE_WMAX];
  int pe[WWAVES];
  int cnt[2 * SF_WIDE_NMAX];      // rows leading at each column (same bit index)
  int16_t lead[SF_WIDE_NMAX];
  int16_t list[SF_WIDE_NMAX];
  double2 amp;
  int nlist, best, piv, pmin, kx, err, ue, tex;
};

namespace wide {

enum { E_OK = 0, E_FORM = 1, E_SUPPORT = 2, E_GATE = 3 };

__device__ __forceinline__ int bitof(const uint64_t* v, int q) { return (int)((v[q >> 6] >> (q & 63)) & 1ull); }

// exponent of i in the product of the literal strings (x1, z1) (x2, z2) on
// one word (Table 1: XY = iZ, YZ = iX, ZX = iY, reversed products -i)
__device__ __forceinline__ int gword(uint64_t a, uint64_t b, uint64_t c, uint64_t d) {
  const uint64_t pos = (a & b & ~c & d) | (a & ~b & c & d) | (~a & b & c & ~d);
  const uint64_t neg = (a & b & c & ~d) | (a & ~b & ~c & d) | (~a & b & c & d);
  return __popcll(pos) - __popcll(neg);
}

// sign bit c of row1 * row2 = (-1)^c (row1 xor row2) for commuting rows
__device__ __forceinline__ int rowsign(const uint64_t* x1, const uint64_t* z1, const uint64_t* x2,
                                      const uint64_t* z2, int W) {
  int e = 0;
  for (int w = 0; w < W; ++w) e += gword(x1[w], z1[w], x2[w], z2[w]);
  return (e & 3) >> 1;
}

__device__ __forceinline__ int row_lead(const uint64_t* x, const uint64_t* z, int W, int n) {
  for (int w = 0; w < W; ++w)
    if (x[w]) return 64 * w + __builtin_ctzll(x[w]);
  for (int w = 0; w < W; ++w)
    if (z[w]) return n + 64 * w + __builtin_ctzll(z[w]);
  return -1;
}

__device__ __forceinline__ int wave_sum(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// i^e as a complex number
__device__ __forceinline__ double2 ipow(int e) {
  e &= 3;
  return make_double2(e == 0 ? 1.0 : e == 2 ? -1.0 : 0.0, e == 1 ? 1.0 : e == 3 ? -1.0 : 0.0);
}

// complex product without fused multiply-add
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(__dsub_rn(__dmul_rn(a.x, b.x), __dmul_rn(a.y, b.y)),
                      __dadd_rn(__dmul_rn(a.x, b.y), __dmul_rn(a.y, b.x)));
}

__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(__dmul_rn(a.x, s), __dmul_rn(a.y, s)); }

struct Frame {
  int n, W;
  int seg, rpw;   // lanes per row (power of two >= W) and rows per wavefront step
  uint64_t* rx;
  uint64_t* rz;
};

// bit index of a lead column: x column q -> q, z column n + q -> 64 W + q
__device__ __forceinline__ int cbit(const Frame F, int col) { return col < F.n ? col : 64 * F.W + (col - F.n); }

// A row's lead changes (by its owning thread): lead counts, X-block size and
// the candidate set follow.
__device__ __forceinline__ void set_lead(WideLds& L, const Frame F, int i, int nl) {
  const int old = L.lead[i];
  if (old == nl) return;
  if (old >= 0) atomicSub(&L.cnt[cbit(F, old)], 1);
  if (nl >= 0) {
    const int b = cbit(F, nl);
    atomicAdd(&L.cnt[b], 1);
    atomicOr((unsigned long long*)&L.cand[b >> 6], 1ull << (b & 63));
  }
  const int dx = (nl >= 0 && nl < F.n) - (old >= 0 && old < F.n);
  if (dx) atomicAdd(&L.kx, dx);
  L.lead[i] = (int16_t)nl;
}

// Add to the candidates the bits of v (word w of the candidate index) that
// are lead columns.
__device__ __forceinline__ void add_lead_bits(WideLds& L, int w, uint64_t v) {
  uint64_t keep = 0;
  while (v) {
    const int b = __builtin_ctzll(v);
    v &= v - 1;
    if (L.cnt[64 * w + b] > 0) keep |= 1ull << b;
  }
  if (keep) atomicOr((unsigned long long*)&L.cand[w], keep);
}

// Full scan of one row's lead (one thread).
__device__ int row_lead_scan(const Frame F, int i) {
  const uint64_t* X = F.rx + (size_t)i * F.W;
  const uint64_t* Z = F.rz + (size_t)i * F.W;
  for (int w = 0; w < F.W; ++w)
    if (X[w]) return 64 * w + __builtin_ctzll(X[w]);
  for (int w = 0; w < F.W; ++w)
    if (Z[w]) return F.n + 64 * w + __builtin_ctzll(Z[w]);
  return -1;
}

// Multiply row m into every row of L.list[0..nlist) except m (lanes over
// words, rows in aligned lane segments): signs into sigma, leads and the
// candidates follow; rows that leave the X-block put their z bits in zpend.
__device__ void absorb(WideLds& L, const Frame F, int m) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = F.n, W = F.W, seg = F.seg, rpw = F.rpw;
  const int r = lane / seg, w = lane % seg, l0 = r * seg;
  const uint64_t smask = (seg == 64 ? ~0ull : ((1ull << seg) - 1)) << l0;
  const uint64_t xm = w < W ? F.rx[(size_t)m * W + w] : 0ull;
  const uint64_t zm = w < W ? F.rz[(size_t)m * W + w] : 0ull;
  const int sm = bitof(L.sig, m);
  const int nh = L.nlist;
  // KP row groups per step, their words loaded up front
  constexpr int KP = 4;
  const int stride = WWAVES * rpw;
  for (int j0 = wv * rpw; j0 < nh; j0 += KP * stride) {
    uint64_t xs[KP], zs[KP];
#pragma unroll
    for (int t = 0; t < KP; ++t) {
      const int j = j0 + t * stride + r;
      const int i = j < nh ? L.list[j] : m;
      const bool ok = j < nh && i != m && w < W;
      xs[t] = ok ? F.rx[(size_t)i * W + w] : 0ull;
      zs[t] = ok ? F.rz[(size_t)i * W + w] : 0ull;
    }
#pragma unroll
    for (int t = 0; t < KP; ++t) {
      const int j = j0 + t * stride + r;
      const int i = j < nh ? L.list[j] : m;
      const bool act = j < nh && i != m;
      const bool ok = act && w < W;
      const int old = L.lead[i];
      const uint64_t x = xs[t], z = zs[t];
      int e = ok ? gword(x, z, xm, zm) : 0;
      for (int o = seg >> 1; o > 0; o >>= 1) e += __shfl_xor(e, o);
      const uint64_t nx = x ^ xm, nz = z ^ zm;
      if (ok) { F.rx[(size_t)i * W + w] = nx; F.rz[(size_t)i * W + w] = nz; }
      const uint64_t xb = __ballot(ok && nx != 0ull) & smask;
      const uint64_t zb = __ballot(ok && nz != 0ull) & smask;
      const int myc = xb ? (nx ? __builtin_ctzll(nx) : 64) : (nz ? __builtin_ctzll(nz) : 64);
      const int src = xb ? __builtin_ctzll(xb) : zb ? __builtin_ctzll(zb) : lane;
      const int c = __shfl(myc, src);
      const bool toz = act && old < n && xb == 0ull;
      if (ok && toz && nz) atomicOr((unsigned long long*)&L.zpend[w], nz);
      if (act && lane == l0) {
        const int nl = xb ? 64 * (src - l0) + c : zb ? n + 64 * (src - l0) + c : -1;
        set_lead(L, F, i, nl);
        if (sm ^ ((e & 3) >> 1)) atomicXor((unsigned long long*)&L.sig[i >> 6], 1ull << (i & 63));
      }
    }
  }
}

// Rows with a bit at column col (z columns: Z-block rows only, unless all)
// into L.list; L.piv = lowest slot leading at col, L.pmin = lowest slot in
// the list.
__device__ void collect(WideLds& L, const Frame F, int col, bool all) {
  const int tid = threadIdx.x, n = F.n, W = F.W;
  if (tid == 0) { L.nlist = 0; L.piv = 0x7fffffff; L.pmin = 0x7fffffff; }
  __syncthreads();
  const bool xcol = col < n;
  const int q = xcol ? col : col - n;
  const uint64_t* base = (xcol ? F.rx : F.rz) + (q >> 6);
  constexpr int KR = 4;
  for (int c0 = 0; c0 < n; c0 += KR * WT) {
    uint64_t wv[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = c0 + tid + WT * k;
      wv[k] = i < n ? base[(size_t)i * W] : 0ull;
    }
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = c0 + tid + WT * k;
      if (i >= n) break;
      const int ld = L.lead[i];
      if (((wv[k] >> (q & 63)) & 1ull) && (xcol || all || ld >= n)) {
        L.list[atomicAdd(&L.nlist, 1)] = (int16_t)i;
        atomicMin(&L.pmin, i);
        if (ld == col) atomicMin(&L.piv, i);
      }
    }
  }
  __syncthreads();
}

// After row m was multiplied into the rows with a bit at an x column (xcol)
// or into Z-block rows with a bit at a z column: the changed rows gained m's
// bits, so the lead columns among them are candidates -- for an x column only
// m's x bits count (the changed rows stay in the X-block, whose z bits are
// free) plus the z bits of rows that left the X-block.
__device__ void add_row_candidates(WideLds& L, const Frame F, int m, bool xcol) {
  const int tid = threadIdx.x, W = F.W;
  __syncthreads();
  if (tid < W) {
    const uint64_t v = xcol ? F.rx[(size_t)m * W + tid] : 0ull;
    if (v) add_lead_bits(L, tid, v);
  } else if (tid < 2 * W) {
    const uint64_t v = (xcol ? 0ull : F.rz[(size_t)m * W + tid - W]) | L.zpend[tid - W];
    if (v) add_lead_bits(L, tid, v);
  }
  __syncthreads();
  if (tid < W) L.zpend[tid] = 0ull;
}

// Repair the form: take the smallest candidate column that rows lead at; if
// another row of its block has a bit there, multiply the lowest slot leading
// there into every such row.  New bits appear only at larger columns, so the
// candidates are taken in increasing order and each column is handled once.
__device__ void repair(WideLds& L, const Frame F) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int W = F.W;
  for (int guard = 0; guard <= 2 * F.n + 2; ++guard) {
    __syncthreads();
    if (tid < 64) {
      // lowest candidate bit that is a lead column (others are dropped)
      int pick = 0x7fffffff;
      for (;;) {
        const uint64_t v = lane < 2 * W ? L.cand[lane] : 0ull;
        const uint64_t nzw = __ballot(v != 0ull);
        if (!nzw) break;
        const int w0 = __builtin_ctzll(nzw);
        const uint64_t vw = L.cand[w0];
        const int b = 64 * w0 + __builtin_ctzll(vw);
        if (lane == 0) L.cand[w0] = vw & (vw - 1);
        __builtin_amdgcn_wave_barrier();
        if (L.cnt[b] > 0) { pick = b; break; }
      }
      if (lane == 0) L.best = pick;
    }
    __syncthreads();
    const int b = L.best;
    if (b == 0x7fffffff || L.err) return;
    const int col = b < 64 * W ? b : F.n + (b - 64 * W);
    collect(L, F, col, false);
    const int m = L.piv;
    if (L.nlist <= 1 || m == 0x7fffffff) continue;
    absorb(L, F, m);
    add_row_candidates(L, F, m, col < F.n);
  }
  if (tid == 0) atomicOr(&L.err, 1 << E_FORM);
  __syncthreads();
}

// Amplitude of psi(M, sigma) at L.s relative to b*: the X-block rows whose
// x-leads are set in s multiply to P with P |b*> ~ |s>.  Sets L.bst = b* =
// s ^ x(P) and L.ue = e with psi(s) = 2^{-k/2} i^e.
__device__ void walk(WideLds& L, const Frame F) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = F.n, W = F.W;
  if (tid == 0) L.nlist = 0;
  __syncthreads();
  for (int i = tid; i < n; i += WT) {
    const int ld = L.lead[i];
    if (ld >= 0 && ld < n && bitof(L.s, ld)) L.list[atomicAdd(&L.nlist, 1)] = (int16_t)i;
  }
  __syncthreads();
  const int m = L.nlist;
  uint64_t ax = 0, az = 0;
  int e = 0, sg = 0;
  for (int j = wv; j < m; j += WWAVES) {
    const int i = L.list[j];
    const uint64_t x = lane < W ? F.rx[(size_t)i * W + lane] : 0ull;
    const uint64_t z = lane < W ? F.rz[(size_t)i * W + lane] : 0ull;
    e += gword(ax, az, x, z);
    ax ^= x;
    az ^= z;
    sg ^= bitof(L.sig, i);
  }
  e = wave_sum(e);
  if (lane < W) { L.px[wv][lane] = ax; L.pz[wv][lane] = az; }
  if (lane == 0) L.pe[wv] = e + 2 * sg;
  __syncthreads();
  if (wv == 0) {
    uint64_t bx = lane < W ? L.px[0][lane] : 0ull, bz = lane < W ? L.pz[0][lane] : 0ull;
    int f = 0;
    for (int v = 1; v < WWAVES; ++v) {
      const uint64_t x = lane < W ? L.px[v][lane] : 0ull, z = lane < W ? L.pz[v][lane] : 0ull;
      f += gword(bx, bz, x, z);
      bx ^= x;
      bz ^= z;
    }
    const uint64_t b = lane < W ? (L.s[lane] ^ bx) : 0ull;
    // P = i^G X^x Z^z in literal form: P |b> = i^{G + |x & z|} (-1)^{z . b} |b ^ x>
    f += __popcll(bx & bz) + 2 * (__popcll(bz & b) & 1);
    f = wave_sum(f);
    if (lane < W) L.bst[lane] = b;
    if (lane == 0) {
      int tot = f;
      for (int v = 0; v < WWAVES; ++v) tot += L.pe[v];
      L.ue = tot & 3;
    }
  }
  __syncthreads();
}

// b* against the form and the signs: zero at every x-lead (by construction)
// and z_h . b* = sigma_h on every Z-block row h, which holds exactly when the
// walk's string lay in the support.  Rows in lane segments.
__device__ void check_support(WideLds& L, const Frame F) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = F.n, W = F.W, seg = F.seg, rpw = F.rpw;
  const int r = lane / seg, w = lane % seg, l0 = r * seg;
  const uint64_t smask = (seg == 64 ? ~0ull : ((1ull << seg) - 1)) << l0;
  for (int i0 = wv * rpw; i0 < n; i0 += WWAVES * rpw) {
    const int i = i0 + r;
    const bool zrow = i < n && L.lead[i] >= n;
    const uint64_t z = zrow && w < W ? F.rz[(size_t)i * W + w] : 0ull;
    const int par = __popcll(__ballot(__popcll(z & (w < W ? L.bst[w] : 0ull)) & 1) & smask) & 1;
    if (zrow && lane == l0 && par != bitof(L.sig, i)) atomicOr(&L.err, 1 << E_SUPPORT);
  }
  __syncthreads();
}

// Table 2 on the columns of the gate's qubits: row i's bits at a (and b)
// change and its sign flip goes into sigma.  Its lead follows from the old
// one unless the old lead sat on a changed column (then the row is scanned);
// the changed columns and every new lead become repair candidates.
__device__ void conjugate(WideLds& L, const Frame F, int op, int a, int b) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = F.n, W = F.W;
  const int wa = a >> 6, wb = b >> 6;
  const uint64_t ma = 1ull << (a & 63), mb = 1ull << (b & 63);
  const bool two = op == DG_CNOT || op == DG_CZ;
  // rows i = tid + WT k in chunks of KR per thread, the gate's words of a
  // chunk loaded up front
  constexpr int KR = 4;
  for (int c0 = 0; c0 < n; c0 += KR * WT) {
  uint64_t pXa[KR], pZa[KR], pXb[KR], pZb[KR];
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int i = c0 + tid + WT * k;
    const bool ok = i < n;
    pXa[k] = ok ? F.rx[(size_t)i * W + wa] : 0ull;
    pZa[k] = ok ? F.rz[(size_t)i * W + wa] : 0ull;
    pXb[k] = ok && two ? F.rx[(size_t)i * W + wb] : 0ull;
    pZb[k] = ok && two ? F.rz[(size_t)i * W + wb] : 0ull;
  }
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int i0 = c0 + WT * k;
    if (i0 >= n) break;
    const int i = i0 + tid;
    int flip = 0;
    if (i < n) {
      uint64_t* X = F.rx + (size_t)i * W;
      uint64_t* Z = F.rz + (size_t)i * W;
      const uint64_t Xa = pXa[k], Za = pZa[k];
      const uint64_t Xb = pXb[k], Zb = pZb[k];
      const int xa = (Xa & ma) != 0, za = (Za & ma) != 0;
      const int xb = (Xb & mb) != 0, zb = (Zb & mb) != 0;
      uint64_t tXa = 0, tZa = 0, tXb = 0, tZb = 0;   // bits to toggle in words a, b
      switch (op) {
        case DG_H: flip = xa & za; if (xa != za) { tXa = ma; tZa = ma; } break;
        case DG_S: flip = xa & za; if (xa) tZa = ma; break;
        case DG_SDG: flip = xa & (za ^ 1); if (xa) tZa = ma; break;
        case DG_X: flip = za; break;
        case DG_Z: flip = xa; break;
        case DG_Y: flip = xa ^ za; break;
        case DG_CNOT:
          flip = xa & zb & (xb ^ za ^ 1);
          if (xa) tXb = mb;
          if (zb) tZa = ma;
          break;
        case DG_CZ:
          flip = xa & xb & (za ^ zb);
          if (xb) tZa = ma;
          if (xa) tZb = mb;
          break;
      }
      if (tXa | tZa | tXb | tZb) {
        if (wa == wb && two) {
          X[wa] = Xa ^ tXa ^ tXb;
          Z[wa] = Za ^ tZa ^ tZb;
        } else {
          if (tXa | tZa) { X[wa] = Xa ^ tXa; Z[wa] = Za ^ tZa; }
          if (tXb | tZb) { X[wb] = Xb ^ tXb; Z[wb] = Zb ^ tZb; }
        }
        const int old = L.lead[i];
        const int nxa = xa ^ (tXa != 0), nxb = two ? (xb ^ (tXb != 0)) : 0;
        const int nza = za ^ (tZa != 0), nzb = two ? (zb ^ (tZb != 0)) : 0;
        int nl;
        if (old == a || old == n + a || (two && (old == b || old == n + b))) {
          nl = row_lead_scan(F, i);
          if (old < n && (nl < 0 || nl >= n))
            for (int w = 0; w < W; ++w)
              if (Z[w]) atomicOr((unsigned long long*)&L.zpend[w], Z[w]);
        } else if (old < n) {
          nl = old;
          if (nxa && a < nl) nl = a;
          if (nxb && b < nl) nl = b;
        } else {
          int xl = 0x7fffffff;
          if (nxa) xl = a;
          if (nxb && b < xl) xl = b;
          if (xl != 0x7fffffff) {
            nl = xl;
          } else {
            nl = old;
            if (nza && n + a < nl) nl = n + a;
            if (nzb && n + b < nl) nl = n + b;
          }
        }
        set_lead(L, F, i, nl);
      }
    }
    const uint64_t fm = __ballot(flip);
    if (lane == 0 && i0 + 64 * wv < n) L.sig[(i0 >> 6) + wv] ^= fm;
  }
  }
  if (tid < (two ? 4 : 2)) {
    const int col = tid == 0 ? a : tid == 1 ? n + a : tid == 2 ? b : n + b;
    const int bb = cbit(F, col);
    atomicOr((unsigned long long*)&L.cand[bb >> 6], 1ull << (bb & 63));
  }
  __syncthreads();
  if (tid < W) {
    add_lead_bits(L, W + tid, L.zpend[tid]);
    L.zpend[tid] = 0ull;
  }
  __syncthreads();
}

// One Clifford gate with its phase factor.
__device__ void clifford(WideLds& L, const Frame F, int op, int a, int b) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int n = F.n, W = F.W;
  const double r2 = 0.70710678118654752440;
  const int ba = bitof(L.bst, a), bb = (op == DG_CNOT || op == DG_CZ) ? bitof(L.bst, b) : 0;
  const int k0 = L.kx;
  double2 beta;
  if (op == DG_H) {
    // old amplitude at b* ^ e_a: nonzero only if an X-block row is X or Y on a alone
    if (tid == 0) { L.piv = -1; L.tex = -1; }
    __syncthreads();
    for (int i = tid; i < n; i += WT)
      if (L.lead[i] == a) L.piv = i;
    __syncthreads();
    const int l = L.piv;
    if (l >= 0 && tid < 64) {
      const uint64_t x = lane < W ? F.rx[(size_t)l * W + lane] : 0ull;
      const uint64_t z = lane < W ? F.rz[(size_t)l * W + lane] : 0ull;
      const uint64_t want = lane == (a >> 6) ? (1ull << (a & 63)) : 0ull;
      const uint64_t bw = lane < W ? L.bst[lane] : 0ull;
      const bool single = __ballot(lane < W && x != want) == 0ull;
      const int par = __popcll(__ballot(__popcll(z & bw) & 1)) & 1;
      const int za = __popcll(__ballot(lane == (a >> 6) && ((z >> (a & 63)) & 1ull)));
      if (lane == 0 && single) L.tex = (2 * (bitof(L.sig, l) ^ par) + za) & 3;
    }
    __syncthreads();
    // A[c] = 2^{k/2} psi(b* with bit a = c): A[ba] = 1 (b* itself), A[ba ^ 1] = t
    const int te = L.tex;
    const int tre = te < 0 ? 0 : (te == 0 ? 1 : te == 2 ? -1 : 0);
    const int tim = te < 0 ? 0 : (te == 1 ? 1 : te == 3 ? -1 : 0);
    // <c|H psi> = r2 (A[0] + (-1)^c A[1]); take c with a nonzero value
    int sre = 1 + tre, sim = tim, c = 0;
    if (sre == 0 && sim == 0) {
      sre = ba ? tre - 1 : 1 - tre;
      sim = ba ? tim : -tim;
      c = 1;
    }
    beta = make_double2(__dmul_rn(r2, (double)sre), __dmul_rn(r2, (double)sim));
    for (int w = tid; w < W; w += WT) {
      uint64_t v = L.bst[w];
      if (w == (a >> 6)) v = (v & ~(1ull << (a & 63))) | ((uint64_t)c << (a & 63));
      L.s[w] = v;
    }
  } else {
    int e = 0;
    switch (op) {
      case DG_S: e = ba; break;
      case DG_SDG: e = 3 * ba; break;
      case DG_Z: e = 2 * ba; break;
      case DG_Y: e = 1 + 2 * ba; break;
      case DG_CZ: e = 2 * (ba & bb); break;
      default: e = 0;
    }
    beta = ipow(e);
    for (int w = tid; w < W; w += WT) {
      uint64_t v = L.bst[w];
      if ((op == DG_X || op == DG_Y) && w == (a >> 6)) v ^= 1ull << (a & 63);
      if (op == DG_CNOT && ba && w == (b >> 6)) v ^= 1ull << (b & 63);
      L.s[w] = v;
    }
  }
  __syncthreads();
  // S, S-dagger and CZ change z bits of X-block rows only, and Paulis change
  // signs only: the form holds.  H and CNOT can break it.
  if (op == DG_H || op == DG_CNOT) {
    conjugate(L, F, op, a, b);
    repair(L, F);
  } else {
    conjugate(L, F, op, a, b);
    if (tid < 2 * W) L.cand[tid] = 0ull;
  }
  walk(L, F);
  if (tid == 0) {
    const int dk = L.kx - k0;
    double2 om = beta;
    if (dk == 1) om = cscale(om, sqrt(2.0));
    else if (dk == -1) om = cscale(om, sqrt(0.5));
    else if (dk != 0) atomicOr(&L.err, 1 << E_FORM);
    om = cmul(om, ipow(-L.ue));
    L.amp = cmul(L.amp, om);
  }
  __syncthreads();
}

__device__ __forceinline__ uint64_t splitmix(uint64_t state, uint64_t index) {
  uint64_t z = state + (index + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Z measurement of qubit q with the seeded coin of measurement index mi.
__device__ void measure(WideLds& L, const Frame F, const WideJob& J, int q, int mi, uint64_t seed) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int n = F.n, W = F.W;
  const double r2 = 0.70710678118654752440;
  const double u = (double)(splitmix(seed, (uint64_t)mi) >> 11) * (1.0 / 9007199254740992.0);
  collect(L, F, q, true);
  const int p = L.pmin;
  if (p == 0x7fffffff) {
    // Z_q is the Z-block row leading at z column q; its sign is the outcome
    if (tid == 0) L.best = -1;
    __syncthreads();
    for (int i = tid; i < n; i += WT)
      if (L.lead[i] == n + q) L.best = i;
    __syncthreads();
    const int h = L.best;
    if (tid == 0) {
      if (h < 0) {
        atomicOr(&L.err, 1 << E_FORM);
      } else {
        const int x = bitof(L.sig, h);
        const double m2 = __dadd_rn(__dmul_rn(L.amp.x, L.amp.x), __dmul_rn(L.amp.y, L.amp.y));
        const double p1 = x ? m2 : 0.0, p0 = x ? 0.0 : m2;
        const int o = u < p1 ? 1 : 0;
        const double po = o ? p1 : p0;
        const double sc = po > 0.0 ? 1.0 / sqrt(po) : 0.0;
        if (fabs(u - p1) < 1e-12 || po <= 0.0) atomicOr(J.flags, 1);
        J.outcomes[mi] = (uint8_t)o;
        J.pvals[mi] = p1;
        L.amp = cscale(L.amp, sc);
      }
    }
    __syncthreads();
    return;
  }
  // random: row p anticommutes with Z_q.  Old amplitude at b* ^ x_p:
  // g_p |b*> = (-1)^{sigma_p + z_p . b*} i^{|x_p & z_p|} |b* ^ x_p>.
  if (tid < 64) {
    const uint64_t x = lane < W ? F.rx[(size_t)p * W + lane] : 0ull;
    const uint64_t z = lane < W ? F.rz[(size_t)p * W + lane] : 0ull;
    const uint64_t b = lane < W ? L.bst[lane] : 0ull;
    const int par = __popcll(__ballot(__popcll(z & b) & 1)) & 1;
    const int yy = wave_sum(__popcll(x & z));
    if (lane == 0) L.tex = (2 * (bitof(L.sig, p) ^ par) + yy) & 3;
  }
  if (tid == 0) {
    const double cr = __dmul_rn(L.amp.x, r2), ci = __dmul_rn(L.amp.y, r2);
    const double m2 = __dadd_rn(__dmul_rn(cr, cr), __dmul_rn(ci, ci));
    const int o = u < m2 ? 1 : 0;
    if (fabs(u - m2) < 1e-12 || m2 <= 0.0) atomicOr(J.flags, 1);
    J.outcomes[mi] = (uint8_t)o;
    J.pvals[mi] = m2;
    L.best = o;
  }
  __syncthreads();
  const int o = L.best;
  const int x0 = bitof(L.bst, q);
  const int ae = o == x0 ? 0 : L.tex;   // old amplitude at the child's string, 2^{-k/2} i^ae
  for (int w = tid; w < W; w += WT) L.s[w] = L.bst[w] ^ (o == x0 ? 0ull : F.rx[(size_t)p * W + w]);
  __syncthreads();
  // the other rows with an x bit at q absorb row p
  absorb(L, F, p);
  add_row_candidates(L, F, p, true);
  // row p becomes (-1)^o Z_q
  for (int w = tid; w < W; w += WT) {
    F.rx[(size_t)p * W + w] = 0ull;
    F.rz[(size_t)p * W + w] = w == (q >> 6) ? (1ull << (q & 63)) : 0ull;
  }
  if (tid == 0) {
    set_lead(L, F, p, n + q);
    const uint64_t m = 1ull << (p & 63);
    L.sig[p >> 6] = o ? (L.sig[p >> 6] | m) : (L.sig[p >> 6] & ~m);
  }
  __syncthreads();
  repair(L, F);
  walk(L, F);
  if (tid == 0) {
    // c_o = a i^ae conj(u') / sqrt 2, then renormalised by 1 / sqrt(p)
    const double cr = __dmul_rn(L.amp.x, r2), ci = __dmul_rn(L.amp.y, r2);
    const double m2 = __dadd_rn(__dmul_rn(cr, cr), __dmul_rn(ci, ci));
    const double sc = m2 > 0.0 ? 1.0 / sqrt(m2) : 0.0;
    double2 c = cmul(L.amp, ipow(ae - L.ue));
    c = cscale(c, r2);
    L.amp = cscale(c, sc);
  }
  __syncthreads();
}

}  // namespace wide

// Device gates [g0, g1) of one frame, by the whole workgroup.
__device__ void wide_body(WideLds& L, const WideJob& J) {
  WideHdr* H = (WideHdr*)J.base;
  const int tid = threadIdx.x;
  const int n = H->n, W = H->W;
  if (n < 1 || n > SF_WIDE_NMAX || W != (n + 63) / 64) return;
  const WideLayout o = wide_layout(n);
  wide::Frame F;
  F.n = n;
  F.W = W;
  F.seg = 1;
  while (F.seg < W) F.seg <<= 1;
  F.rpw = 64 / F.seg;
  F.rx = (uint64_t*)(J.base + o.rx);
  F.rz = (uint64_t*)(J.base + o.rz);
  const uint64_t* gsig = (const uint64_t*)(J.base + o.sig);
  const uint64_t* gbst = (const uint64_t*)(J.base + o.bst);
  int32_t* glead = (int32_t*)(J.base + o.lead);
  for (int w = tid; w < W; w += WT) { L.sig[w] = gsig[w]; L.bst[w] = gbst[w]; L.zpend[w] = 0ull; }
  for (int w = tid; w < 2 * W; w += WT) L.cand[w] = 0ull;
  for (int c = tid; c < 128 * W; c += WT) L.cnt[c] = 0;
  if (tid == 0) {
    L.amp = H->amp;
    L.kx = 0;
    L.err = H->error;
  }
  const uint64_t seed = H->seed;
  int nm = H->nmeas;
  __syncthreads();
  for (int i = tid; i < n; i += WT) {
    const int ld = glead[i];
    L.lead[i] = (int16_t)ld;
    if (ld >= 0 && ld < 2 * n) atomicAdd(&L.cnt[wide::cbit(F, ld)], 1);
    if (ld >= 0 && ld < n) atomicAdd(&L.kx, 1);
  }
  __syncthreads();
  for (int gi = J.g0; gi < J.g1; ++gi) {
    if (L.err) break;
    const DGate g = J.gates[gi];
    if (g.op == DG_MEASURE) {
      if (g.q0 < 0 || g.q0 >= n) { if (tid == 0) L.err |= 1 << wide::E_GATE; __syncthreads(); break; }
      wide::measure(L, F, J, g.q0, nm, seed);
      ++nm;
    } else if (g.op >= 0 && g.op < DG_NCPHASE) {
      const bool two = g.op == DG_CNOT || g.op == DG_CZ;
      if (g.q0 < 0 || g.q0 >= n || (two && (g.q1 < 0 || g.q1 >= n || g.q1 == g.q0))) {
        if (tid == 0) L.err |= 1 << wide::E_GATE;
        __syncthreads();
        break;
      }
      wide::clifford(L, F, g.op, g.q0, two ? g.q1 : 0);
    } else {
      if (tid == 0) L.err |= 1 << wide::E_GATE;
      __syncthreads();
      break;
    }
  }
  __syncthreads();
  if (J.g1 > J.g0 && !L.err) wide::check_support(L, F);
  uint64_t* sig = (uint64_t*)(J.base + o.sig);
  uint64_t* bst = (uint64_t*)(J.base + o.bst);
  for (int w = tid; w < W; w += WT) { sig[w] = L.sig[w]; bst[w] = L.bst[w]; }
  for (int i = tid; i < n; i += WT) glead[i] = L.lead[i];
  if (tid == 0) {
    H->amp = L.amp;
    H->k = L.kx;
    H->nmeas = nm;
    H->error = L.err;
  }
}

// Many frames (blockIdx.x = frame).
extern "C" __global__ void __launch_bounds__(WT) sf_wide_run(const WideJob* __restrict__ jobs) {
  __shared__ WideLds L;
  const WideJob J = jobs[blockIdx.x];
  wide_body(L, J);
}

extern "C" __global__ void __launch_bounds__(WT) sf_wide_one(WideJob job) {
  __shared__ WideLds L;
  wide_body(L, job);
}

// Basis state |b>: row q = Z_q with sign b_q, b* = b, a = 1.
extern "C" __global__ void __launch_bounds__(WT) sf_wide_init(unsigned char* base, int n, const uint64_t* basis,
                                                              uint64_t seed, int* flags) {
  WideHdr* H = (WideHdr*)base;
  const int W = (n + 63) / 64;
  const WideLayout o = wide_layout(n);
  uint64_t* rx = (uint64_t*)(base + o.rx);
  uint64_t* rz = (uint64_t*)(base + o.rz);
  uint64_t* sig = (uint64_t*)(base + o.sig);
  uint64_t* bst = (uint64_t*)(base + o.bst);
  int32_t* lead = (int32_t*)(base + o.lead);
  for (size_t t = threadIdx.x; t < (size_t)n * W; t += WT) {
    const size_t i = t / W, w = t % W;
    rx[t] = 0ull;
    rz[t] = w == (i >> 6) ? (1ull << (i & 63)) : 0ull;
  }
  for (int w = threadIdx.x; w < W; w += WT) {
    uint64_t v = basis ? basis[w] : 0ull;
    if (w == W - 1 && (n & 63)) v &= (1ull << (n & 63)) - 1;
    sig[w] = v;
    bst[w] = v;
  }
  for (int i = threadIdx.x; i < n; i += WT) lead[i] = n + i;
  if (threadIdx.x == 0) {
    uint64_t* hw = (uint64_t*)H;
    for (int w = 0; w < (int)(sizeof(WideHdr) / 8); ++w) hw[w] = 0ull;
    H->n = n;
    H->W = W;
    H->amp = make_double2(1.0, 0.0);
    H->seed = seed;
    *flags = 0;
  }
}

// Canonical readout: X-block rows lose their z bits at Z-block leads (each
// Z-block row whose lead they hit is multiplied in, replayed on sigma), then
// rows are ordered by lead, which gives the fully reduced row echelon form
// with rows sorted by pivot.  out: tableau (n rows of [x words | z words]),
// then sigma (W words), then the amplitude (2 doubles); work: 2 n W words.
extern "C" __global__ void __launch_bounds__(WT) sf_wide_readout(const unsigned char* base, uint64_t* out,
                                                                 uint64_t* work) {
  __shared__ uint64_t sig[SF_WIDE_WMAX], zlm[SF_WIDE_WMAX], lm[2 * SF_WIDE_WMAX], osig[SF_WIDE_WMAX];
  __shared__ int16_t zrow[SF_WIDE_NMAX], lead[SF_WIDE_NMAX];
  __shared__ int err;
  const WideHdr* H = (const WideHdr*)base;
  const int n = H->n, W = H->W, tid = threadIdx.x;
  if (n < 1 || n > SF_WIDE_NMAX) return;
  const WideLayout o = wide_layout(n);
  const uint64_t* rx = (const uint64_t*)(base + o.rx);
  const uint64_t* rz = (const uint64_t*)(base + o.rz);
  const int32_t* glead = (const int32_t*)(base + o.lead);
  uint64_t* wx = work;
  uint64_t* wz = work + (size_t)n * W;
  for (size_t t = tid; t < (size_t)n * W; t += WT) { wx[t] = rx[t]; wz[t] = rz[t]; }
  for (int w = tid; w < W; w += WT) { sig[w] = ((const uint64_t*)(base + o.sig))[w]; zlm[w] = 0; osig[w] = 0; }
  for (int w = tid; w < 2 * W; w += WT) lm[w] = 0;
  for (int i = tid; i < n; i += WT) { lead[i] = (int16_t)glead[i]; zrow[i] = -1; }
  if (tid == 0) err = 0;
  __syncthreads();
  for (int i = tid; i < n; i += WT) {
    const int ld = lead[i];
    if (ld < 0 || ld >= 2 * n) { atomicOr(&err, 1); continue; }
    atomicOr((unsigned long long*)&lm[ld >> 6], 1ull << (ld & 63));
    if (ld >= n) {
      zrow[ld - n] = (int16_t)i;
      atomicOr((unsigned long long*)&zlm[(ld - n) >> 6], 1ull << ((ld - n) & 63));
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += WT) {
    const int ld = lead[i];
    if (ld < 0 || ld >= n) continue;
    uint64_t* X = wx + (size_t)i * W;
    uint64_t* Z = wz + (size_t)i * W;
    int fl = 0;
    for (int w = 0; w < W; ++w) {
      uint64_t m = Z[w] & zlm[w];
      while (m) {
        const int q = 64 * w + __builtin_ctzll(m);
        m &= m - 1;
        const int h = zrow[q];
        const uint64_t* Xh = wx + (size_t)h * W;
        const uint64_t* Zh = wz + (size_t)h * W;
        const int c = wide::rowsign(X, Z, Xh, Zh, W);
        for (int v = 0; v < W; ++v) { X[v] ^= Xh[v]; Z[v] ^= Zh[v]; }
        fl ^= wide::bitof(sig, h) ^ c;
      }
    }
    if (fl) atomicXor((unsigned long long*)&sig[i >> 6], 1ull << (i & 63));
  }
  __syncthreads();
  for (int i = tid; i < n; i += WT) {
    const int ld = lead[i];
    if (ld < 0 || ld >= 2 * n) continue;
    int pos = 0;
    for (int w = 0; w < (ld >> 6); ++w) pos += __popcll(lm[w]);
    pos += __popcll(lm[ld >> 6] & ((1ull << (ld & 63)) - 1));
    for (int w = 0; w < W; ++w) {
      out[(size_t)pos * 2 * W + w] = wx[(size_t)i * W + w];
      out[(size_t)pos * 2 * W + W + w] = wz[(size_t)i * W + w];
    }
    if (wide::bitof(sig, i)) atomicOr((unsigned long long*)&osig[pos >> 6], 1ull << (pos & 63));
  }
  __syncthreads();
  uint64_t* os = out + (size_t)n * 2 * W;
  for (int w = tid; w < W; w += WT) os[w] = osig[w];
  if (tid == 0) {
    double2* oa = (double2*)(os + W);
    *oa = err ? make_double2(0.0, 0.0) : H->amp;
  }
}
