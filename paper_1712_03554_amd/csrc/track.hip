// Tableau track (one wavefront per frame, everything in LDS).
//
// For each gate of a circuit range this kernel
//   * conjugates the stabilizer matrix (Table 2) and collects the per-row sign
//     flips, which ROTATE applies to every phase vector (section 3);
//   * restores the row-echelon form (Invariant 1) by Gaussian elimination
//     restricted to the columns the gate disturbed, recording each row
//     multiplication and replaying it on the hull (s0, V) of the phase vectors;
//   * derives the per-element global-phase factor of the gate (the five-step
//     global-phase algorithm of section 3) as a function of the hull
//     coordinates, by evaluating it at 1 + d + d(d-1)/2 coordinate vectors and
//     fitting the quadratic form that it is;
//   * for a non-Clifford phase gate or a measurement, performs COFACTOR
//     (section 3): forced-outcome measurement of the tableau, the child map of
//     every phase vector, and the amplitude factor of each cofactor.
// The results are per-segment programs (SegProg) that the element kernels in
// elem.hip apply to the amplitude array.
//
// For frames of up to 128 qubits the work is split over three kernels: the
// track kernel walks the gates in order doing only what must be sequential
// (the tableau update, the echelon repair with its replay on the hull, the
// cofactors) and records the state after every gate; the phase kernel then
// evaluates every Clifford gate's phase factor at the fitting points from the
// records before and after it, one wavefront per gate, all gates at once; the
// fit kernel sums each segment's factors and fits its quadratic form.  Wider
// frames (TrkL) do all of it in the track kernel.
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "sf_dev.h"

#define TL 64  // one wavefront

// LDS of one tableau-track workgroup.  NM row slots of WM words in the
// row-indexed arrays (rows, column copy, pre-gate rows, b* basis, indexes);
// the hull and sample arrays are sized for the largest frames.
//
// The fields up to (not including) cx are all the phase kernel uses: it
// allocates only that prefix (phase_lds_bytes), which lets more of its
// wavefronts share a compute unit.
template <int NM, int WM>
struct LdsT {
  static constexpr int RN = NM, RW = WM;
  uint64_t rx[NM * WM], rz[NM * WM];
  uint64_t ox[NM * WM], oz[NM * WM];
  uint64_t beta[NM * WM];
  uint64_t s0[SF_WMAX], V[SF_DMAX][SF_WMAX], u[SF_WMAX];
  uint64_t os0[SF_WMAX], oV[SF_DMAX][SF_WMAX];
  uint64_t hbO[SF_DMAX + 2][SF_WMAX], hbN[SF_DMAX + 2][SF_WMAX];
  uint64_t oxpm[SF_WMAX];
  uint64_t zsm[SF_WMAX];           // slot mask of Z-block slots
  uint64_t tc[16];                // per-phase shader clocks
  uint32_t Ys[SF_PMAX];
  int misc[8];                    // [0] X-block size, [1] last lead stamp
  int16_t lead[NM], xpiv[NM], zpiv[NM], oxpiv[NM];
  uint8_t ow[NM];
  uint8_t t0[SF_PMAX];
  // -- track kernel only from here --
  uint64_t cx[NM * WM], cz[NM * WM];   // column q: slots with an x (z) bit at q
  uint64_t rmask[SF_WMAX], cmask[SF_WMAX], fmask[SF_WMAX];
  uint64_t dq[SF_WMAX];
  uint8_t acc[SF_PMAX], t1[SF_PMAX];
  uint32_t ech[SF_DMAX];          // scratch for span tests
  uint32_t lst[2 * NM];           // lead stamps of the elimination passes
};

// LDS bytes of the phase kernel: the prefix of LdsT before the track-only fields
template <class LT>
constexpr size_t phase_lds_bytes() { return offsetof(LT, cx); }

typedef LdsT<SF_NMAX, SF_WMAX> Lds;

typedef Lds TrackLdsProbe;

// phases: 0 save, 1 column update, 2 repair, 3 index+b* images, 4 sampling,
// 5 fitting, 6 cofactor, 7 total, 8 repair checks, 9 repair row products,
// 10 repair replay on the hull, 11 elimination passes (a count), 12 pivot
// index, 13 b* basis, 14 hull images, 15 sample points evaluated (a count)
// (compiled in with -DSF_TRACK_TIMERS; each reading waits for outstanding LDS
// traffic, so the counters are off in normal builds)
#ifdef SF_TRACK_TIMERS
#define TIC(k) do { if (lane_id() == 0) L.tc[k] -= clock64(); } while (0)
#define TOC(k) do { if (lane_id() == 0) L.tc[k] += clock64(); } while (0)
#define TCLOCK() clock64()
#else
#define TIC(k) do { } while (0)
#define TOC(k) do { } while (0)
#define TCLOCK() 0ull
#endif

__device__ __forceinline__ int getb(const uint64_t* v, int q) { return (int)((v[q >> 6] >> (q & 63)) & 1ull); }
__device__ __forceinline__ void flipb(uint64_t* v, int q) { v[q >> 6] ^= 1ull << (q & 63); }
__device__ __forceinline__ int par64(uint64_t v) { return __popcll(v) & 1; }

template <class LT>
__device__ __forceinline__ int colbit(const LT& L, int i, int col, int n) {
  return col < n ? getb(&L.rx[i * LT::RW], col) : getb(&L.rz[i * LT::RW], col - n);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x; }

// Global-memory view of a pointer.  Accesses through a generic pointer become
// flat instructions, which count against the LDS wait counter as well: every
// LDS wait of the gate loop would then also wait for the record stores and
// the next gate's prefetch.  Through these the compiler emits global
// instructions, which only the vector-memory counter tracks.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ DGate load_gate(const DGate* p) {
  auto q = gmem(p);
  DGate g;
  g.op = q->op;
  g.q0 = q->q0;
  g.q1 = q->q1;
  g.q2 = q->q2;
  g.c = q->c;
  g.s = q->s;
  return g;
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int s) {
  const int lo = __shfl_xor((int)(uint32_t)v, s);
  const int hi = __shfl_xor((int)(uint32_t)(v >> 32), s);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// 64 x 64 bit transpose across the wavefront: on entry lane r holds row r
// (bit c = entry (r, c)), on exit lane c holds column c (bit r = entry
// (r, c)).  Six butterfly stages swap the off-diagonal blocks of 32, 16, ...,
// 1 bits between lanes r and r ^ s.  Every lane must take part.
__device__ __forceinline__ uint64_t transpose64(uint64_t v) {
  const int lane = lane_id();
  const uint64_t masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                             0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    const int s = 32 >> t;
    const uint64_t m = masks[t];
    const uint64_t p = shfl_xor64(v, s);
    v = (lane & s) ? (((p >> s) & m) | (v & ~m)) : ((v & m) | ((p & m) << s));
  }
  return v;
}

// (every lane holds the maximum after the butterfly; reading it from lane 0
// tells the compiler that the result is wave-uniform, so branches and loop
// exits that depend on it stay scalar)
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) {
    int t = __shfl_xor(v, o);
    v = t > v ? t : v;
  }
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int pair_index(int j, int jj, int d) {
  return 1 + d + (j * (2 * d - j - 1)) / 2 + (jj - j - 1);
}

template <class LT>
__device__ void build_points(LT& L, int d) {
  const int lane = lane_id();
  if (lane == 0) L.Ys[0] = 0;
  for (int j = lane; j < d; j += TL) {
    L.Ys[1 + j] = 1u << j;
    for (int jj = j + 1; jj < d; ++jj) L.Ys[pair_index(j, jj, d)] = (1u << j) | (1u << jj);
  }
  __syncthreads();
}

__device__ __forceinline__ int npoints(int d) { return 1 + d + d * (d - 1) / 2; }

// fit e(Y) mod 4 from samples f at the points (must be a Z4 quadratic form)
template <class LT>
__device__ void fit_z4(LT& L, const uint8_t* f, int d, Z4Q* out, int* err) {
  const int lane = lane_id();
  uint32_t q = 0;
  int l = 0;
  if (lane < d) {
    l = (f[1 + lane] - f[0]) & 3;
    for (int jj = lane + 1; jj < d; ++jj) {
      int v = (f[pair_index(lane, jj, d)] - f[1 + lane] - f[1 + jj] + f[0]) & 3;
      if (v & 1) *err = TRK_E_INTERNAL;
      q |= (uint32_t)(v >> 1) << jj;
    }
  }
  uint32_t L1 = (uint32_t)__ballot(lane < d && (l & 1));
  uint32_t L2 = (uint32_t)__ballot(lane < d && (l >> 1));
  uint32_t qnz = (uint32_t)__ballot(lane < d && q != 0);
  auto o = gmem(out);
  if (lane < 32) o->Q[lane] = lane < d ? q : 0u;
  if (lane == 0) { o->c = f[0] & 3; o->L1 = L1; o->L2 = L2; o->qnz = qnz; }
}

template <class LT>
__device__ void fit_gf2(LT& L, const uint8_t* t, int d, GF2Q* out) {
  const int lane = lane_id();
  uint32_t q = 0;
  int l = 0;
  if (lane < d) {
    l = (t[1 + lane] ^ t[0]) & 1;
    for (int jj = lane + 1; jj < d; ++jj)
      q |= (uint32_t)((t[pair_index(lane, jj, d)] ^ t[1 + lane] ^ t[1 + jj] ^ t[0]) & 1) << jj;
  }
  uint32_t Lm = (uint32_t)__ballot(lane < d && l);
  uint32_t qnz = (uint32_t)__ballot(lane < d && q != 0);
  auto o = gmem(out);
  if (lane < 32) o->Q[lane] = lane < d ? q : 0u;
  if (lane == 0) { o->c = t[0] & 1; o->L = Lm; o->qnz = qnz; o->pad = 0; }
}

__device__ void zero_z4(Z4Q* out) {
  const int lane = lane_id();
  auto o = gmem(out);
  if (lane < 32) o->Q[lane] = 0;
  if (lane == 0) { o->c = 0; o->L1 = 0; o->L2 = 0; o->qnz = 0; }
}

__device__ void emit_header(SegProg* out, int kind, int is_meas, int d, int d_out, int nhad, int had_off) {
  auto sp = gmem(out);
  sp->kind = kind; sp->is_meas = is_meas; sp->d = d; sp->d_out = d_out;
  sp->nhad = nhad; sp->had_off = had_off; sp->nhad_total = nhad;
  sp->j0 = -1; sp->delta = 0; sp->det_c = 0; sp->det_r = 0;
  sp->m_c0 = 0; sp->m_r = 0; sp->m_j0 = -1; sp->meas_index = -1; sp->pad = 0;
  sp->det2_c = 0; sp->det2_r = 0;
  sp->ph_re = 1.0; sp->ph_im = 0.0;
}

// qubit value functional of a deterministic qubit q: sigma bit of the Z-row
// that equals Z_q, as a function of Y
template <class LT>
__device__ void apply_pending(LT& L, const TrackState* st, const uint8_t* outcomes, int* dptr) {
  const int lane = lane_id();
  int d = *dptr;
  int o = outcomes ? (int)outcomes[st->pend_meas] : 0;
  int bsel = o ^ st->pend_c0;
  uint32_t r = st->pend_r;
  int j0 = st->pend_j0;
  if (r != 0) {
    uint64_t vj0[SF_WMAX];
    for (int w = 0; w < SF_WMAX; ++w) vj0[w] = L.V[j0][w];
    __syncthreads();
    if (lane == 0 && bsel) for (int w = 0; w < SF_WMAX; ++w) L.s0[w] ^= vj0[w];
    uint64_t mine[SF_WMAX];
    if (lane < d)
      for (int w = 0; w < SF_WMAX; ++w) mine[w] = L.V[lane][w] ^ (((r >> lane) & 1u) ? vj0[w] : 0ull);
    __syncthreads();
    if (lane < d && lane != j0) {
      int dst = lane < j0 ? lane : lane - 1;
      for (int w = 0; w < SF_WMAX; ++w) L.V[dst][w] = mine[w];
    }
    d -= 1;
    __syncthreads();
  }
  *dptr = d;
}


template <int W>
struct Trk {
// LDS sized for this word count: 64 W row slots of W words
typedef LdsT<64 * W, W> LL;

// The tableau as the Clifford loop keeps it: lane l holds row slots and
// columns 64k + l (k < W); rows x/z (W words each), the column-major copy
// cx/cz (slot masks of rows with an x / z bit at that qubit) and each row's
// lead column.  LDS holds write-only snapshots of it for random access.
struct Regs {
  uint64_t x[W][W], z[W][W], cx[W][W], cz[W][W];
  int ld[W];
};

static __device__ __forceinline__ uint64_t pick(const uint64_t (&v)[W], int w) {
  uint64_t r = 0;
  for (int t = 0; t < W; ++t) if (t == w) r = v[t];
  return r;
}

static __device__ __forceinline__ uint64_t bcast64(uint64_t v, int l) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
}

static __device__ __forceinline__ void regs_load(const LL& L, Regs& R, int n) {
  const int lane = lane_id();
  for (int k = 0; k < W; ++k) {
    const int i = 64 * k + lane;
    const bool ok = i < n;
    for (int w = 0; w < W; ++w) {
      R.x[k][w] = ok ? L.rx[i * LL::RW + w] : 0ull;
      R.z[k][w] = ok ? L.rz[i * LL::RW + w] : 0ull;
      R.cx[k][w] = ok ? L.cx[i * LL::RW + w] : 0ull;
      R.cz[k][w] = ok ? L.cz[i * LL::RW + w] : 0ull;
    }
    R.ld[k] = ok ? (int)L.lead[i] : -1;
  }
}

// rows, leads and (cols) the column-major copy into LDS; no barrier
static __device__ __forceinline__ void regs_store(LL& L, const Regs& R, int n, bool cols) {
  const int lane = lane_id();
  for (int k = 0; k < W; ++k) {
    const int i = 64 * k + lane;
    if (i >= n) continue;
    for (int w = 0; w < W; ++w) {
      L.rx[i * LL::RW + w] = R.x[k][w];
      L.rz[i * LL::RW + w] = R.z[k][w];
      if (cols) {
        L.cx[i * LL::RW + w] = R.cx[k][w];
        L.cz[i * LL::RW + w] = R.cz[k][w];
      }
    }
    L.lead[i] = (int16_t)R.ld[k];
  }
}

static __device__ int row_lead(const uint64_t* x, const uint64_t* z, int n) {
  for (int w = 0; w < W; ++w) if (x[w]) return 64 * w + __builtin_ctzll(x[w]);
  for (int w = 0; w < W; ++w) if (z[w]) return n + 64 * w + __builtin_ctzll(z[w]);
  return -1;
}

// The same with selects instead of branches (register rows of every lane).
static __device__ __forceinline__ int row_lead_sel(const uint64_t (&x)[W], const uint64_t (&z)[W], int n) {
  int ld = -1;
  for (int w = W - 1; w >= 0; --w) ld = z[w] ? n + 64 * w + (int)__builtin_ctzll(z[w]) : ld;
  for (int w = W - 1; w >= 0; --w) ld = x[w] ? 64 * w + (int)__builtin_ctzll(x[w]) : ld;
  return ld;
}

// Sign bit c of row1 * row2 = (-1)^c (row1 xor row2) for commuting rows,
// from the literal products of Table 1 (XY=iZ, YZ=iX, ZX=iY; reversed -i).
static __device__ int rowprod_sign(const uint64_t* x1, const uint64_t* z1, const uint64_t* x2,
                            const uint64_t* z2) {
  int pos = 0, neg = 0;
  for (int w = 0; w < W; ++w) {
    uint64_t a = x1[w], b = z1[w], c = x2[w], d = z2[w];
    pos += __popcll((a & b & ~c & d) | (a & ~b & c & d) | (~a & b & c & ~d));
    neg += __popcll((a & b & c & ~d) | (a & ~b & ~c & d) | (~a & b & c & d));
  }
  return ((pos - neg) & 3) >> 1;
}

// ---------------------------------------------------------------------------
// Echelon bookkeeping
// ---------------------------------------------------------------------------
static __device__ void rebuild_index(LL& L, int n) {
  const int lane = lane_id();
  for (int i = lane; i < LL::RN; i += TL) { L.xpiv[i] = -1; L.zpiv[i] = -1; }
  __syncthreads();
  for (int i = lane; i < n; i += TL) {
    int ld = row_lead(&L.rx[i * LL::RW], &L.rz[i * LL::RW], n);
    L.lead[i] = (int16_t)ld;
    if (ld >= 0 && ld < n) L.xpiv[ld] = (int16_t)i;
    else if (ld >= n) L.zpiv[ld - n] = (int16_t)i;
  }
  __syncthreads();
  const int R = (n + 63) / 64;
  int k = 0;
  for (int it = 0; it < R; ++it) {
    int i = it * 64 + lane;
    bool isx = i < n && L.lead[i] >= 0 && L.lead[i] < n;
    bool isz = i < n && L.lead[i] >= n;
    uint64_t bx = __ballot(isx), bz = __ballot(isz);
    k += __popcll(bx);
    if (lane == 0) L.zsm[it] = bz;
  }
  if (lane == 0) {
    for (int it = R; it < SF_WMAX; ++it) L.zsm[it] = 0;
    L.misc[0] = k;
  }
  __syncthreads();
}

// Tracked phase-vector images: s0 (affine), V[0..d) and optionally u (linear).
// Apply sigma_i ^= sigma_m ^ c_i for every i in rmask (c in cmask).
static __device__ void apply_rowsum_batch(LL& L, int m, int d, bool with_u) {
  const int lane = lane_id();
  uint64_t* vec = nullptr;
  bool affine = false;
  if (lane < d) vec = L.V[lane];
  else if (lane == d) { vec = L.s0; affine = true; }
  else if (lane == d + 1 && with_u) vec = L.u;
  if (vec) {
    int bm = getb(vec, m);
    for (int w = 0; w < W; ++w) vec[w] ^= (bm ? L.rmask[w] : 0ull) ^ (affine ? L.cmask[w] : 0ull);
  }
  __syncthreads();
}

// rows in L.rmask received row m: toggle those slots in every column where
// row m has a bit
static __device__ void cols_rowsum(LL& L, int m, int n) {
  const int lane = lane_id();
  const int R = (n + 63) / 64;
  for (int it = 0; it < R; ++it) {
    const int q = it * 64 + lane;
    if (q >= n) continue;
    if (getb(&L.rx[m * LL::RW], q))
      for (int w = 0; w < W; ++w) L.cx[q * LL::RW + w] ^= L.rmask[w];
    if (getb(&L.rz[m * LL::RW], q))
      for (int w = 0; w < W; ++w) L.cz[q * LL::RW + w] ^= L.rmask[w];
  }
}

// Gaussian elimination restricted to the columns that break the echelon
// form: a column breaks it when it is the lead of some row and at least two
// rows have a bit there (on z columns only Z-block rows count, unless full).
// full = 0 keeps the form of Figure 2b (X-block reduced on x-leads, Z-block
// reduced on z-leads); full = 1 also clears X-block bits on z-leads.  Each
// step takes the smallest such column, multiplies its first leading row into
// every other row with a bit there, and replays the row multiplication on the
// tracked phase vectors.
// Rows, their leads, the column-major copy and the tracked phase vectors are
// held in registers for the whole loop: lane l owns
// row slots and columns 64k + l (k < W) and hull vector l (V[l], then s0 at
// lane d, u at lane d + 1).  The pivot row travels by readlane, the row masks
// of each step by ballot; LDS is read on entry and written on exit only.
static __device__ __forceinline__ void repair_core(LL& L, Regs& R, uint64_t (&hv)[W], uint32_t& gen, int n, int d,
                                                   bool with_u, int full) {
  const int lane = lane_id();
  uint64_t (&x)[W][W] = R.x;
  uint64_t (&z)[W][W] = R.z;
  uint64_t (&cxr)[W][W] = R.cx;
  uint64_t (&czr)[W][W] = R.cz;
  int (&ld)[W] = R.ld;
  bool valid[W];
  for (int k = 0; k < W; ++k) valid[k] = 64 * k + lane < n;
  const bool has_vec = lane < d || lane == d || (lane == d + 1 && with_u);
  const bool affine = lane == d;
  for (int guard = 0; guard < 4 * SF_NMAX + 8; ++guard) {
#ifdef SF_TRACK_TIMERS
    if (lane == 0) L.tc[11] += 1;  // elimination passes
#endif
    TIC(8);
    // Z-block rows (no x bits)
    uint64_t zs[W];
    for (int k = 0; k < W; ++k) {
      uint64_t xa = 0;
      for (int w = 0; w < W; ++w) xa |= x[k][w];
      const uint64_t b = __ballot(valid[k] && xa == 0ull);
      zs[k] = full ? ~0ull : b;
    }
    // every row stamps its lead column; a column breaks the form if it holds
    // this pass's stamp and at least two bits (z columns: Z-block rows only
    // unless full).  The smallest such column, x columns before z columns.
    ++gen;
    for (int k = 0; k < W; ++k)
      if (valid[k] && ld[k] >= 0) L.lst[ld[k]] = gen;
    __syncthreads();
    uint64_t px[W], pz[W];
    // (all stamps are read at once: q < 64 W and n + q < 2 * 64 W are in
    // range for every lane, so no read waits on a condition)
    uint32_t sx[W], sz[W];
    for (int k = 0; k < W; ++k) {
      sx[k] = L.lst[64 * k + lane];
      sz[k] = L.lst[n + 64 * k + lane];
    }
    for (int k = 0; k < W; ++k) {
      const int q = 64 * k + lane;
      int a = 0, b = 0;
      for (int w = 0; w < W; ++w) { a += __popcll(cxr[k][w]); b += __popcll(czr[k][w] & zs[w]); }
      const bool ok = q < n;
      px[k] = __ballot(ok & (a >= 2) & (sx[k] == gen));
      pz[k] = __ballot(ok & (b >= 2) & (sz[k] == gen));
    }
    int col = -1;
    for (int k = 0; k < W; ++k) if (col < 0 && px[k]) col = 64 * k + __builtin_ctzll(px[k]);
    for (int k = 0; k < W; ++k) if (col < 0 && pz[k]) col = n + 64 * k + __builtin_ctzll(pz[k]);
    TOC(8);
    if (col < 0) break;
    TIC(9);
    // pivot: the first slot leading at col
    int m = -1;
    for (int k = 0; k < W && m < 0; ++k) {
      const uint64_t b = __ballot(valid[k] && ld[k] == col);
      if (b) m = 64 * k + __builtin_ctzll(b);
    }
    const int km = m >> 6, lm = m & 63;
    uint64_t xm[W], zm[W];
    for (int w = 0; w < W; ++w) {
      uint64_t sx = 0, sz = 0;
      for (int kk = 0; kk < W; ++kk)
        if (kk == km) { sx = x[kk][w]; sz = z[kk][w]; }
      xm[w] = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(sx >> 32), lm) << 32) |
              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)sx, lm);
      zm[w] = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(sz >> 32), lm) << 32) |
              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)sz, lm);
    }
    int wm = 0;
    for (int w = 0; w < W; ++w) wm += __popcll(xm[w] & zm[w]);
    const bool xcol = col < n;
    const int cb = xcol ? col : col - n;
    uint64_t rm[W], cm[W];
    for (int k = 0; k < W; ++k) {
      const int i = 64 * k + lane;
      uint64_t xa = 0, wsel = 0;
      for (int w = 0; w < W; ++w) {
        xa |= x[k][w];
        if ((cb >> 6) == w) wsel = xcol ? x[k][w] : z[k][w];
      }
      const bool hit = valid[k] & (i != m) & (xcol | (full != 0) | (xa == 0ull)) & (((wsel >> (cb & 63)) & 1ull) != 0);
      // P(x1,z1) P(x2,z2) = i^e P(x1^x2, z1^z2) with
      // e = |x1 z1| + |x2 z2| + 2 |z1 x2| - |(x1^x2)(z1^z2)|  (Y = iXZ);
      // for commuting rows e is even and the sign is (-1)^(e/2).  Every
      // lane computes the product; the hit rows take it.
      int e = wm;
      uint64_t nx[W], nz[W];
      for (int w = 0; w < W; ++w) {
        nx[w] = x[k][w] ^ xm[w];
        nz[w] = z[k][w] ^ zm[w];
        e += __popcll(x[k][w] & z[k][w]) + 2 * __popcll(z[k][w] & xm[w]) - __popcll(nx[w] & nz[w]);
      }
      const int c = (e & 3) >> 1;
      const int nl = row_lead_sel(nx, nz, n);
      for (int w = 0; w < W; ++w) {
        x[k][w] = hit ? nx[w] : x[k][w];
        z[k][w] = hit ? nz[w] : z[k][w];
      }
      ld[k] = hit ? nl : ld[k];
      rm[k] = __ballot(hit);
      cm[k] = __ballot(hit & (c != 0));
    }
    // the column-major copy: columns where row m has a bit get the hit rows
    for (int k = 0; k < W; ++k) {
      if (!valid[k]) continue;
      const bool bx = (xm[k] >> lane) & 1ull, bz = (zm[k] >> lane) & 1ull;
      for (int w = 0; w < W; ++w) {
        if (bx) cxr[k][w] ^= rm[w];
        if (bz) czr[k][w] ^= rm[w];
      }
    }
    TOC(9);
    TIC(10);
    // replay on the tracked phase vectors: sigma_i ^= sigma_m (^ c_i on s0)
    if (has_vec) {
      uint64_t wm = 0;
      for (int w = 0; w < W; ++w) if ((m >> 6) == w) wm = hv[w];
      const bool bm = (wm >> (m & 63)) & 1ull;
      for (int w = 0; w < W; ++w) hv[w] ^= (bm ? rm[w] : 0ull) ^ (affine ? cm[w] : 0ull);
    }
    TOC(10);
  }
}

// The same on the LDS copy of the tableau, hull and stamp generation
// (terminal steps and readout).
static __device__ void repair(LL& L, int n, int d, bool with_u, int full) {
  const int lane = lane_id();
  Regs R;
  regs_load(L, R, n);
  uint64_t hv[W];
  for (int w = 0; w < W; ++w)
    hv[w] = lane < d ? L.V[lane][w] : lane == d ? L.s0[w] : (lane == d + 1 && with_u) ? L.u[w] : 0ull;
  uint32_t gen = (uint32_t)L.misc[1];
  repair_core(L, R, hv, gen, n, d, with_u, full);
  regs_store(L, R, n, true);
  if (lane < d) for (int w = 0; w < W; ++w) L.V[lane][w] = hv[w];
  else if (lane == d) for (int w = 0; w < W; ++w) L.s0[w] = hv[w];
  else if (lane == d + 1 && with_u) for (int w = 0; w < W; ++w) L.u[w] = hv[w];
  if (lane == 0) L.misc[1] = (int)gen;
  __syncthreads();
}

// ---------------------------------------------------------------------------
// b*(sigma): smallest basis string of the support of psi(M, sigma).
// Flipping the sign of Z-block row h moves the support by e_{q_h} (X_{q_h}
// anticommutes with that row only); the result is then reduced on the X-block
// leads.  So b*(sigma) = XOR over Z-rows h with sigma_h = 1 of beta_h, with
// beta_h = e_{q_h} ^ (x-part of the X-row leading at q_h, if any).
// ---------------------------------------------------------------------------
static __device__ void build_beta(LL& L, int n) {
  const int lane = lane_id();
  for (int h = lane; h < n; h += TL) {
    uint64_t* b = &L.beta[h * LL::RW];
    for (int w = 0; w < W; ++w) b[w] = 0;
    int ld = L.lead[h];
    if (ld >= n) {
      int q = ld - n;
      flipb(b, q);
      int l = L.xpiv[q];
      if (l >= 0)
        for (int w = 0; w < W; ++w) b[w] ^= L.rx[l * LL::RW + w];
    }
  }
  __syncthreads();
}

static __device__ void bimage(const LL& L, const uint64_t* vec, uint64_t* out) {
  uint64_t acc[SF_WMAX] = {0, 0, 0, 0};
  for (int w = 0; w < W; ++w) {
    uint64_t bits = vec[w] & L.zsm[w];
    while (bits) {
      int h = 64 * w + __builtin_ctzll(bits);
      bits &= bits - 1;
      for (int v = 0; v < W; ++v) acc[v] ^= L.beta[h * LL::RW + v];
    }
  }
  for (int w = 0; w < W; ++w) out[w] = acc[w];
}

// images of s0 (index 0), V[j] (1+j) and, if with_u, u (index d+1) into hb
static __device__ void hull_images(LL& L, uint64_t (*hb)[SF_WMAX], int d, bool with_u) {
  const int lane = lane_id();
  if (lane == 0) bimage(L, L.s0, hb[0]);
  else if (lane <= d) bimage(L, L.V[lane - 1], hb[lane]);
  else if (lane == d + 1 && with_u) bimage(L, L.u, hb[d + 1]);
  __syncthreads();
}

// exponent e with psi(M_old, sigma)(b) = 2^{-k/2} i^e, or -1 if b is outside
// the support.  The old X-block rows are stored by pivot column (ox/oz/ow at
// q hold the row whose x-lead is q; oxpiv[q] is its slot, for its sign).  psi ~ prod_l (I + g_l)/2 |b*>: the amplitude at b* ^ x_S is the
// phase of applying the X-block generators in S to |b*>.
static __device__ int uexp(const LL& L, const uint64_t* sig, const uint64_t* bO, const uint64_t* b) {
  uint64_t v[SF_WMAX];
  for (int w = 0; w < W; ++w) v[w] = bO[w];
  int e = 0;
  for (int w = 0; w < W; ++w) {
    uint64_t D = (b[w] ^ bO[w]) & L.oxpm[w];
    // two generators per pass: their rows are read before either is applied
    // (the reads depend on the pivot columns only, not on v)
    while (D) {
      const int q0 = 64 * w + __builtin_ctzll(D);
      D &= D - 1;
      const bool two = D != 0;
      const int q1 = two ? 64 * w + __builtin_ctzll(D) : q0;
      D &= two ? D - 1 : D;
      const int l0 = L.oxpiv[q0], l1 = L.oxpiv[q1];
      const int w0 = L.ow[q0], w1 = L.ow[q1];
      uint64_t oz0[W], ox0[W], oz1[W], ox1[W];
      for (int t = 0; t < W; ++t) {
        oz0[t] = L.oz[q0 * LL::RW + t];
        ox0[t] = L.ox[q0 * LL::RW + t];
        oz1[t] = L.oz[q1 * LL::RW + t];
        ox1[t] = L.ox[q1 * LL::RW + t];
      }
      uint64_t zv = 0;
      for (int t = 0; t < W; ++t) zv ^= oz0[t] & v[t];
      e += 2 * (getb(sig, l0) ^ par64(zv)) + w0;
      for (int t = 0; t < W; ++t) v[t] ^= ox0[t];
      if (two) {
        zv = 0;
        for (int t = 0; t < W; ++t) zv ^= oz1[t] & v[t];
        e += 2 * (getb(sig, l1) ^ par64(zv)) + w1;
        for (int t = 0; t < W; ++t) v[t] ^= ox1[t];
      }
    }
  }
  for (int w = 0; w < W; ++w) if (v[w] != b[w]) return -1;
  return e & 3;
}

// ---------------------------------------------------------------------------
// Sample points and fitting of quadratic forms over the hull coordinates
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Save the pre-gate tableau and hull (needed by the phase evaluation)
// ---------------------------------------------------------------------------
static __device__ void save_old(LL& L, int n, int d) {
  const int lane = lane_id();
  for (int i = lane; i < n; i += TL) {
    const int ld = L.lead[i];
    if (ld >= 0 && ld < n) {
      int c = 0;
      for (int w = 0; w < W; ++w) {
        L.ox[ld * LL::RW + w] = L.rx[i * LL::RW + w];
        L.oz[ld * LL::RW + w] = L.rz[i * LL::RW + w];
        c += __popcll(L.rx[i * LL::RW + w] & L.rz[i * LL::RW + w]);
      }
      L.ow[ld] = (uint8_t)(c & 3);
    }
    L.oxpiv[i] = L.xpiv[i];
  }
  for (int i = n + lane; i < LL::RN; i += TL) L.oxpiv[i] = -1;
  if (lane < d) for (int w = 0; w < SF_WMAX; ++w) L.oV[lane][w] = L.V[lane][w];
  if (lane == d) for (int w = 0; w < SF_WMAX; ++w) L.os0[w] = L.s0[w];
  if (lane <= d + 1) for (int w = 0; w < SF_WMAX; ++w) L.hbO[lane][w] = L.hbN[lane][w];
  __syncthreads();
  for (int it = 0; it < SF_WMAX; ++it) {
    const int q = it * 64 + lane;
    const uint64_t m = __ballot(q < n && L.xpiv[q] >= 0);
    if (lane == 0) L.oxpm[it] = m;
  }
  __syncthreads();
}

// gather the (<= 2) hull vectors of point Y into sigma/b images
static __device__ __forceinline__ void point_vec(const uint64_t* base, const uint64_t (*vecs)[SF_WMAX], uint32_t Y,
                                          int off, uint64_t* out) {
  for (int w = 0; w < W; ++w) out[w] = base[w];
  while (Y) {
    int j = __builtin_ctz(Y);
    Y &= Y - 1;
    for (int w = 0; w < W; ++w) out[w] ^= vecs[j + off][w];
  }
}

// ---------------------------------------------------------------------------
// Clifford gate
// ---------------------------------------------------------------------------
// Table 2 on the register tableau: conjugate every row by the gate, collect
// the sign flips f (applied to every phase vector through s0 ^= f, s0 being
// lane d's hull register) and keep the column-major copy in step.  Registers
// only.
// One gate kind per instantiation, so that the per-row work is straight-line
// code (the gate is dispatched once, by a scalar branch, in conj_regs).
template <int OP>
static __device__ __forceinline__ void conj_rows(Regs& R, uint64_t (&fm)[W], int wa, int ba, int wb, int bb, int n) {
  for (int k = 0; k < W; ++k) {
    const uint64_t xwa = pick(R.x[k], wa), zwa = pick(R.z[k], wa);
    const int xa = (int)((xwa >> ba) & 1ull), za = (int)((zwa >> ba) & 1ull);
    int xb = 0, zb = 0;
    if constexpr (OP == DG_CNOT || OP == DG_CZ) {
      xb = (int)((pick(R.x[k], wb) >> bb) & 1ull);
      zb = (int)((pick(R.z[k], wb) >> bb) & 1ull);
    }
    int fl = 0;
    uint64_t mxa = 0, mza = 0, mxb = 0, mzb = 0;  // bits to toggle at a and b
    if constexpr (OP == DG_H) { fl = xa & za; mxa = mza = (uint64_t)(xa ^ za) << ba; }
    else if constexpr (OP == DG_S) { fl = xa & za; mza = (uint64_t)xa << ba; }
    else if constexpr (OP == DG_SDG) { fl = xa & (za ^ 1); mza = (uint64_t)xa << ba; }
    else if constexpr (OP == DG_X) { fl = za; }
    else if constexpr (OP == DG_Z) { fl = xa; }
    else if constexpr (OP == DG_Y) { fl = xa ^ za; }
    else if constexpr (OP == DG_CNOT) { fl = xa & zb & (xb ^ za ^ 1); mxb = (uint64_t)xa << bb; mza = (uint64_t)zb << ba; }
    else if constexpr (OP == DG_CZ) { fl = xa & xb & (za ^ zb); mza = (uint64_t)xb << ba; mzb = (uint64_t)xa << bb; }
    if constexpr (OP == DG_H || OP == DG_S || OP == DG_SDG || OP == DG_CNOT || OP == DG_CZ) {
      for (int w = 0; w < W; ++w) {
        R.x[k][w] ^= (w == wa ? mxa : 0ull) | (w == wb ? mxb : 0ull);
        R.z[k][w] ^= (w == wa ? mza : 0ull) ^ (w == wb ? mzb : 0ull);
      }
    }
    // only H and CNOT move leads: the diagonal gates change z bits of rows
    // that have an x bit (whose lead is an x column), the Paulis no bits
    if constexpr (OP == DG_H || OP == DG_CNOT)
      R.ld[k] = (mxa | mza | mxb) ? row_lead_sel(R.x[k], R.z[k], n) : R.ld[k];
    fm[k] = __ballot(fl);
  }
}

static __device__ __forceinline__ void conj_regs(Regs& R, uint64_t (&hv)[W], int op, int a, int b, int n, int d) {
  const int lane = lane_id();
  const int wa = a >> 6, ba = a & 63, wb = b >> 6, bb = b & 63;
  uint64_t fm[W];
  switch (op) {
    case DG_H: conj_rows<DG_H>(R, fm, wa, ba, wb, bb, n); break;
    case DG_S: conj_rows<DG_S>(R, fm, wa, ba, wb, bb, n); break;
    case DG_SDG: conj_rows<DG_SDG>(R, fm, wa, ba, wb, bb, n); break;
    case DG_X: conj_rows<DG_X>(R, fm, wa, ba, wb, bb, n); break;
    case DG_Z: conj_rows<DG_Z>(R, fm, wa, ba, wb, bb, n); break;
    case DG_Y: conj_rows<DG_Y>(R, fm, wa, ba, wb, bb, n); break;
    case DG_CNOT: conj_rows<DG_CNOT>(R, fm, wa, ba, wb, bb, n); break;
    default: conj_rows<DG_CZ>(R, fm, wa, ba, wb, bb, n); break;
  }
  // column-major copy
  if (op == DG_H) {
    if (lane == ba)
      for (int k = 0; k < W; ++k)
        if (k == wa)
          for (int w = 0; w < W; ++w) { const uint64_t t = R.cx[k][w]; R.cx[k][w] = R.cz[k][w]; R.cz[k][w] = t; }
  } else if (op == DG_S || op == DG_SDG) {
    if (lane == ba)
      for (int k = 0; k < W; ++k)
        if (k == wa)
          for (int w = 0; w < W; ++w) R.cz[k][w] ^= R.cx[k][w];
  } else if (op == DG_CNOT) {
    // column b of x gets the rows with x at a; column a of z the rows with z at b
    uint64_t cxa[W], czb[W];
    for (int w = 0; w < W; ++w) {
      uint64_t u = 0, v = 0;
      for (int k = 0; k < W; ++k) { if (k == wa) u = R.cx[k][w]; if (k == wb) v = R.cz[k][w]; }
      cxa[w] = bcast64(u, ba);
      czb[w] = bcast64(v, bb);
    }
    for (int k = 0; k < W; ++k)
      for (int w = 0; w < W; ++w) {
        if (k == wb && lane == bb) R.cx[k][w] ^= cxa[w];
        if (k == wa && lane == ba) R.cz[k][w] ^= czb[w];
      }
  } else if (op == DG_CZ) {
    uint64_t cxa[W], cxb[W];
    for (int w = 0; w < W; ++w) {
      uint64_t u = 0, v = 0;
      for (int k = 0; k < W; ++k) { if (k == wa) u = R.cx[k][w]; if (k == wb) v = R.cx[k][w]; }
      cxa[w] = bcast64(u, ba);
      cxb[w] = bcast64(v, bb);
    }
    for (int k = 0; k < W; ++k)
      for (int w = 0; w < W; ++w) {
        if (k == wa && lane == ba) R.cz[k][w] ^= cxb[w];
        if (k == wb && lane == bb) R.cz[k][w] ^= cxa[w];
      }
  }
  if (lane == d)
    for (int w = 0; w < W; ++w) hv[w] ^= fm[w];
}

// ---------------------------------------------------------------------------
// span test: delta with XOR_{j in delta} oV[j] == dq (slot bit vectors), or
// 0xffffffff if dq is outside the span.  Single lane (d <= 30 vectors).
// ---------------------------------------------------------------------------
// Wave-parallel Gaussian elimination over the d vectors vecs[0..d) (one per
// lane).  Returns delta with XOR_{j in delta} vecs[j] == target, or
// 0xffffffff if the target is outside their span; tops[] receives the
// leading-bit positions of the echelon basis (in the order found).
static __device__ uint32_t span_reduce(const uint64_t (*vecs)[SF_WMAX], const uint64_t* target, int d,
                                       int* tops, int* ntops) {
  const int lane = lane_id();
  uint64_t v[W];
  uint32_t c = 0;
  const bool is_t = lane == 63;
  for (int w = 0; w < W; ++w) v[w] = lane < d ? vecs[lane][w] : (is_t && target ? target[w] : 0ull);
  if (lane < d) c = 1u << lane;
  bool used = false;
  int nt = 0;
  for (int round = 0; round < d; ++round) {
    uint64_t any = 0;
    for (int w = 0; w < W; ++w) any |= v[w];
    uint64_t bal = __ballot(lane < d && !used && any != 0ull);
    if (!bal) break;
    const int pl = __builtin_ctzll(bal);
    uint64_t pv[W];
    for (int w = 0; w < W; ++w) pv[w] = __shfl(v[w], pl);
    const uint32_t pc = __shfl(c, pl);
    int top = -1;
    for (int w = W - 1; w >= 0 && top < 0; --w) if (pv[w]) top = 64 * w + 63 - __builtin_clzll(pv[w]);
    if (tops && lane == 0) tops[nt] = top;
    ++nt;
    if (lane == pl) used = true;
    else if (getb(v, top)) {
      for (int w = 0; w < W; ++w) v[w] ^= pv[w];
      c ^= pc;
    }
  }
  if (ntops) *ntops = nt;
  uint64_t tany = 0;
  for (int w = 0; w < W; ++w) tany |= v[w];
  const uint64_t tz = __shfl(tany, 63);
  const uint32_t tc = __shfl(c, 63);
  return tz ? 0xffffffffu : tc;
}

// ---------------------------------------------------------------------------
// Non-Clifford phase gate or measurement on q: COFACTOR (section 3)
// ---------------------------------------------------------------------------
static __device__ void det_functional(LL& L, int q, int n, int d, uint32_t* c0, uint32_t* r, int* err) {
  const int lane = lane_id();
  int h = L.zpiv[q];
  uint32_t rr = 0;
  if (h < 0) { if (lane == 0) *err = TRK_E_INTERNAL; h = 0; }
  else {
    for (int w = 0; w < W; ++w) {
      uint64_t want = (q >> 6) == w ? (1ull << (q & 63)) : 0ull;
      if (L.rz[h * LL::RW + w] != want || L.rx[h * LL::RW + w] != 0ull) *err = TRK_E_INTERNAL;
    }
  }
  rr = (uint32_t)__ballot(lane < d && getb(L.V[lane < d ? lane : 0], h));
  *c0 = (uint32_t)getb(L.s0, h);
  *r = rr;
}

// Filter step of a measurement on the hull: keep sigma(Y) with
// c0 ^ parity(r & Y) == outcome, i.e. fix coordinate j0 and drop it.

// ---------------------------------------------------------------------------
// Last step of a direct controlled phase / Toffoli (Eqs. 2 and 3): after the
// cofactors on the two controls both are deterministic, with values
// f1(Y) = c1 ^ parity(r1 & Y) and f2(Y) = c2 ^ parity(r2 & Y).  DG_CPH2 puts
// the phase on the elements with f1 & f2.  DG_CX2 applies X on q2 to them: X
// leaves the unsigned matrix as it is and flips the signs of the rows with a z
// bit at q2 (mask f), so such an element moves from sigma(Y) to sigma(Y) ^ f
// with the factor omega(Y) = psi(M, sigma(Y))(b*(sigma(Y) ^ f) ^ e_q2), a Z4
// quadratic form in Y (sampled and fitted as for the Clifford gates).  If f
// is in span(V) (f = sum of V[j], j in delta) the element moves to Y ^ delta,
// which has the same control values (f has no bit on the controls' Z rows);
// otherwise the hull grows by the coordinate V[d] = f.
// ---------------------------------------------------------------------------
static __device__ void terminal_controlled(LL& L, const TrackJob& job, const DGate& gt, int seg, int nhad,
                                           int had_base, int n, int* dptr, int* err) {
  const int lane = lane_id();
  int d = *dptr;
  SegProg* sp = job.dry ? nullptr : job.prog + seg;
  if (!job.dry) {
    // (its Clifford phase E is fitted by the fit kernel when the range has
    // Clifford gates; zero until then)
    if (lane == 0) emit_header(sp, SEG_DET2, 0, d, d, nhad, had_base);
    zero_z4(&sp->E);
    __syncthreads();
  }
  uint32_t c1, r1, c2, r2;
  det_functional(L, gt.q0, n, d, &c1, &r1, err);
  det_functional(L, gt.q1, n, d, &c2, &r2, err);
  if (!job.dry && lane == 0) { sp->det_c = c1; sp->det_r = r1; sp->det2_c = c2; sp->det2_r = r2; }
  if (gt.op == DG_CPH2) {
    if (!job.dry) {
      if (lane == 0) { sp->kind = SEG_DET2; sp->ph_re = gt.c; sp->ph_im = gt.s; }
      zero_z4(&sp->B0);
      zero_z4(&sp->B1);
    }
    __syncthreads();
    return;
  }
  const int t = gt.q2;
  const int R = (n + 63) / 64;
  for (int it = 0; it < SF_WMAX; ++it) {
    const int i = it * 64 + lane;
    const uint64_t b = __ballot(it < R && i < n && getb(&L.rz[i * LL::RW], t));
    if (lane == 0) L.dq[it] = b;
  }
  __syncthreads();
  save_old(L, n, d);
  const uint32_t delta = span_reduce(L.oV, L.dq, d, nullptr, nullptr);
  if (!job.dry) {
    // b*(f): the images are linear, so b*(sigma(Y) ^ f) = b*(sigma(Y)) ^ b*(f)
    if (lane == 0) bimage(L, L.dq, L.hbN[d + 1]);
    __syncthreads();
    const int P = npoints(d);
    for (int pt = lane; pt < P; pt += TL) {
      const uint32_t Y = L.Ys[pt];
      uint64_t so[SF_WMAX], bo[SF_WMAX], src[SF_WMAX];
      point_vec(L.os0, L.oV, Y, 0, so);
      point_vec(L.hbO[0], L.hbO, Y, 1, bo);
      for (int w = 0; w < W; ++w) src[w] = bo[w] ^ L.hbN[d + 1][w];
      flipb(src, t);
      const int e = uexp(L, so, bo, src);
      if (e < 0) *err = TRK_E_INTERNAL;
      L.t0[pt] = (uint8_t)(e & 3);
    }
    __syncthreads();
    fit_z4(L, L.t0, d, &sp->B0, err);
    zero_z4(&sp->B1);
    __syncthreads();
  }
  if (delta != 0xffffffffu) {
    if (!job.dry && lane == 0) {
      sp->kind = SEG_CX2P;
      sp->delta = delta;
      sp->j0 = delta ? 31 - __builtin_clz(delta) : -1;
      sp->d_out = d;
    }
  } else {
    if (lane == 0)
      for (int w = 0; w < SF_WMAX; ++w) L.V[d][w] = L.dq[w];
    d += 1;
    if (!job.dry && lane == 0) { sp->kind = SEG_CX2G; sp->d_out = d; }
  }
  __syncthreads();
  *dptr = d;
}

// ---------------------------------------------------------------------------
// Split form: records of the state after every gate, the per-gate phase
// evaluation from two records, and the per-segment sums.
// ---------------------------------------------------------------------------
static __device__ __forceinline__ int count_x(const Regs& R, int n) {
  const int lane = lane_id();
  int k = 0;
  for (int kk = 0; kk < W; ++kk) {
    const int ld = R.ld[kk];
    k += __popcll(__ballot(64 * kk + lane < n && ld >= 0 && ld < n));
  }
  return k;
}

// record r: rows and hull (lane j < d: V[j], lane d: s0) from the registers
static __device__ __forceinline__ void rec_write(const TrackJob& job, int r, const Regs& R, const uint64_t (&hb)[W],
                                                 int n, int d) {
  auto rw = gmem((uint64_t*)(job.rec + (size_t)r * job.rec_stride));
  const int lane = lane_id();
  for (int k = 0; k < W; ++k) {
    const int i = 64 * k + lane;
    if (i < n)
      for (int w = 0; w < W; ++w) {
        rw[i * 2 * W + w] = R.x[k][w];
        rw[i * 2 * W + W + w] = R.z[k][w];
      }
  }
  auto hv = rw + (size_t)n * 2 * W;
  if (lane <= d)
    for (int w = 0; w < W; ++w) hv[(lane == d ? 0 : lane + 1) * W + w] = hb[w];
  if (lane == 0) *gmem((int32_t*)(job.rec + (size_t)r * job.rec_stride + ((size_t)n * 2 * W + (SF_DMAX + 1) * W) * 8)) = d;
}

// the hull between LDS (terminal steps) and the registers of the Clifford
// loop (lane j < d: V[j], lane d: s0)
static __device__ __forceinline__ void hull_to_regs(const LL& L, uint64_t (&hb)[W], int d) {
  const int lane = lane_id();
  for (int w = 0; w < W; ++w) hb[w] = lane < d ? L.V[lane][w] : lane == d ? L.s0[w] : 0ull;
}

static __device__ __forceinline__ void hull_to_lds(LL& L, const uint64_t (&hb)[W], int d) {
  const int lane = lane_id();
  if (lane < d) for (int w = 0; w < W; ++w) L.V[lane][w] = hb[w];
  else if (lane == d) for (int w = 0; w < W; ++w) L.s0[w] = hb[w];
}

static __device__ __forceinline__ int rec_d(const TrackJob& job, int r, int n) {
  const uint64_t* rw = (const uint64_t*)(job.rec + (size_t)r * job.rec_stride);
  return *(const int32_t*)(rw + (size_t)n * 2 * W + (SF_DMAX + 1) * W);
}

// A record held in registers (lane l: row slots l + 64 k, hull entry l), so
// that the phase kernel can fetch the next record while it works on a gate.
struct RecRegs {
  uint64_t x[W][W], z[W][W], h[W];
  int d;
};

static __device__ __forceinline__ void rec_fetch(const TrackJob& job, int r, int n, RecRegs& R) {
  auto rw = gmem((const uint64_t*)(job.rec + (size_t)r * job.rec_stride));
  const int lane = lane_id();
  for (int k = 0; k < W; ++k) {
    const int i = 64 * k + lane;
    for (int w = 0; w < W; ++w) {
      R.x[k][w] = i < n ? rw[i * 2 * W + w] : 0ull;
      R.z[k][w] = i < n ? rw[i * 2 * W + W + w] : 0ull;
    }
  }
  auto hv = rw + (size_t)n * 2 * W;
  for (int w = 0; w < W; ++w) R.h[w] = lane <= SF_DMAX ? hv[lane * W + w] : 0ull;
  R.d = *gmem((const int32_t*)(job.rec + (size_t)r * job.rec_stride + ((size_t)n * 2 * W + (SF_DMAX + 1) * W) * 8));
}

// The phase kernel's view of the current state carried in registers from
// gate to gate: each lane's row leads (row slots lane and 64 + lane), the
// pivot rows of its columns (xpiv at columns lane and 64 + lane), the
// X-block size, and the image of its hull vector (lane 0: s0, lane j: V[j-1]).
struct PhRegs {
  int ld[W], xp[W];
  int k;
  uint64_t hb[SF_WMAX];
};

// Pre-gate view for the basis-amplitude walk, written from registers: the
// X-block rows by pivot column (ox, oz, ow), the pivot map (oxpiv, oxpm), the
// hull (os0, oV) and its images (hbO).  No LDS is read.
static __device__ __forceinline__ void ph_save_old(LL& L, const RecRegs& cur, const PhRegs& pr, int n, int d) {
  const int lane = lane_id();
  for (int k = 0; k < W; ++k) {
    const int i = 64 * k + lane;
    const int ld = pr.ld[k];
    if (i < n && ld >= 0 && ld < n) {
      int c = 0;
      for (int w = 0; w < W; ++w) {
        L.ox[ld * LL::RW + w] = cur.x[k][w];
        L.oz[ld * LL::RW + w] = cur.z[k][w];
        c += __popcll(cur.x[k][w] & cur.z[k][w]);
      }
      L.ow[ld] = (uint8_t)(c & 3);
    }
    L.oxpiv[i] = i < n ? (int16_t)pr.xp[k] : (int16_t)-1;
  }
  if (lane <= d) {
    for (int w = 0; w < SF_WMAX; ++w) {
      const uint64_t v = w < W ? cur.h[w] : 0ull;
      if (lane == 0) L.os0[w] = v;
      else L.oV[lane - 1][w] = v;
      L.hbO[lane][w] = pr.hb[w];
    }
  }
  for (int k = 0; k < SF_WMAX; ++k) {
    const uint64_t m = k < W ? __ballot(64 * k + lane < n && pr.xp[k] >= 0) : 0ull;
    if (lane == 0) L.oxpm[k] = m;
  }
}

// The new state's rows into LDS (the b* basis gathers other lanes' rows).
static __device__ __forceinline__ void ph_put_rows(LL& L, const RecRegs& R) {
  const int lane = lane_id();
  for (int k = 0; k < W; ++k) {
    const int i = 64 * k + lane;
    for (int w = 0; w < W; ++w) {
      L.rx[i * LL::RW + w] = R.x[k][w];
      L.rz[i * LL::RW + w] = R.z[k][w];
    }
  }
}

// Row leads from the registers, the pivot map by scatter (X-block leads),
// the Z-block slot mask and the X-block size; then each lane's columns'
// pivot rows gathered back.  (rebuild_index without re-reading the rows.)
static __device__ __forceinline__ void ph_index(LL& L, const RecRegs& R, PhRegs& pr, int n) {
  const int lane = lane_id();
  for (int k = 0; k < W; ++k) L.xpiv[64 * k + lane] = -1;
  __syncthreads();
  int kx = 0;
  for (int k = 0; k < W; ++k) {
    const int i = 64 * k + lane;
    const int ld = i < n ? row_lead_sel(R.x[k], R.z[k], n) : -1;
    pr.ld[k] = ld;
    if (ld >= 0 && ld < n) L.xpiv[ld] = (int16_t)i;
    kx += __popcll(__ballot(ld >= 0 && ld < n));
    const uint64_t bz = __ballot(ld >= n);
    if (lane == 0) L.zsm[k] = bz;
  }
  if (lane == 0) for (int k = W; k < SF_WMAX; ++k) L.zsm[k] = 0;
  pr.k = kx;
  __syncthreads();
  for (int k = 0; k < W; ++k) pr.xp[k] = L.xpiv[64 * k + lane];
}

// b* basis rows of the lane's Z-block rows (build_beta with the leads in
// registers).
static __device__ __forceinline__ void ph_beta(LL& L, const PhRegs& pr, int n) {
  const int lane = lane_id();
  for (int k = 0; k < W; ++k) {
    const int h = 64 * k + lane;
    if (h >= n) continue;
    uint64_t b[W];
    for (int w = 0; w < W; ++w) b[w] = 0;
    const int ld = pr.ld[k];
    if (ld >= n) {
      const int q = ld - n;
      b[q >> 6] ^= 1ull << (q & 63);
      const int l = L.xpiv[q];
      if (l >= 0)
        for (int w = 0; w < W; ++w) b[w] ^= L.rx[l * LL::RW + w];
    }
    for (int w = 0; w < W; ++w) L.beta[h * LL::RW + w] = b[w];
  }
  __syncthreads();
}

// Images of the hull vectors (lane j's vector from the record registers)
// into hbN and the lane's register copy.
static __device__ __forceinline__ void ph_images(LL& L, const RecRegs& R, PhRegs& pr, int d) {
  const int lane = lane_id();
  uint64_t out[SF_WMAX] = {0, 0, 0, 0};
  if (lane <= d) {
    bimage(L, R.h, out);
    for (int w = 0; w < SF_WMAX; ++w) L.hbN[lane][w] = out[w];
  }
  for (int w = 0; w < SF_WMAX; ++w) pr.hb[w] = out[w];
  __syncthreads();
}

// The whole new-state view from one record (chunk start, after a terminal
// step, after a non-diagonal gate).
static __device__ __forceinline__ void ph_load(LL& L, const RecRegs& R, PhRegs& pr, int n, int d) {
  ph_put_rows(L, R);
  ph_index(L, R, pr, n);
  ph_beta(L, pr, n);
  ph_images(L, R, pr, d);
}

// segment s starts: its sums start at zero
static __device__ __forceinline__ void seg_clear(const TrackJob& job, int s, int d) {
  if (s >= job.nseg) return;
  const int P = min(npoints(d), job.pe);
  for (int p = lane_id(); p < P; p += TL) *gmem(job.segacc + (size_t)s * job.pe + p) = 0u;
}

// Clifford gate of the split form: Table 2 and the echelon repair only.
// Returns whether the gate is a Hadamard that keeps the support size (a GF(2)
// term of the segment); kx carries the X-block size.
static __device__ __forceinline__ bool clifford_gate_rec(LL& L, Regs& R, uint64_t (&hv)[W], uint32_t& gen, int op,
                                                         int a, int b, int n, int d, int* kx) {
  TIC(1);
  conj_regs(R, hv, op, a, b, n, d);
  TOC(1);
  // the diagonal gates keep the echelon form, the Paulis change signs only
  if (op != DG_H && op != DG_CNOT) return false;
  TIC(2);
  repair_core(L, R, hv, gen, n, d, false, 0);
  TOC(2);
  // CNOT keeps the rank of the x part, so the X-block size
  if (op != DG_H) return false;
  const int knew = count_x(R, n);
  const bool hs = knew == *kx;
  *kx = knew;
  return hs;
}

// Phase factors of the Clifford gates g0 + i, i in [c k, (c + 1) k) with
// k = pchunk, of a split-form range at the fitting points (the evaluation of
// the five-step procedure from the states before and after each gate), added
// into their segments' sums.  The wavefront builds the pivot index, b* basis
// and hull images from the record before its first gate and then carries
// them, with the record itself, in registers (PhRegs, RecRegs): a
// non-diagonal gate writes them out as its pre-gate view and rebuilds from
// the record after it; a diagonal gate changes only z bits of X-block rows
// and X-block signs, which leave the index, the b* basis and the images as
// they are, so only the register copy of the record changes; after a
// terminal step everything is rebuilt.
static __device__ void phase_body(LL& L, const TrackJob& job, int c) {
  const int lane = lane_id();
  const int len = job.g1 - job.g0;
  const int k = job.pchunk > 0 ? job.pchunk : 1;
  const int i0 = c * k;
  if (i0 >= len) return;
  const int i1 = min(len, i0 + k);
  TrackState* st = job.st;
  const int n = __builtin_amdgcn_readfirstlane(st->n);
  int err = 0;
  RecRegs pf;
  rec_fetch(job, i0, n, pf);
  int d = __builtin_amdgcn_readfirstlane(pf.d);
  if (d < 0 || d >= SF_DMAX) {
    if (lane == 0) st->error = TRK_E_INTERNAL;
    return;
  }
  RecRegs cur = pf;   // the state before the next gate
  PhRegs pr;
  ph_load(L, cur, pr, n, d);
  rec_fetch(job, i0 + 1, n, pf);
  build_points(L, d);
  // gate i and its info, fetched one gate ahead like the records
  DGate gnext = load_gate(job.gates + job.g0 + i0);
  int snext = *gmem(job.ginfo + 2 * i0), hnext = *gmem(job.ginfo + 2 * i0 + 1);
  for (int i = i0; i < i1 && !err; ++i) {
    // nx: the record after gate i; the one after gate i + 1 loads meanwhile
    const RecRegs nx = pf;
    const DGate gt = gnext;
    const int sg = snext, hg = hnext;
    if (i + 1 < i1) {
      rec_fetch(job, i + 2, n, pf);
      gnext = load_gate(job.gates + job.g0 + i + 1);
      snext = *gmem(job.ginfo + 2 * (i + 1));
      hnext = *gmem(job.ginfo + 2 * (i + 1) + 1);
    }
    const int op = __builtin_amdgcn_readfirstlane(gt.op);
    const int a = __builtin_amdgcn_readfirstlane(gt.q0), b = __builtin_amdgcn_readfirstlane(gt.q1);
    const int dn = __builtin_amdgcn_readfirstlane(nx.d);
    if (op >= DG_NCPHASE) {
      // terminal step: the next gate starts from the record after it
      if (i + 1 < i1) {
        if (dn < 0 || dn >= SF_DMAX) { err = TRK_E_INTERNAL; break; }
        d = dn;
        cur = nx;
        ph_load(L, cur, pr, n, d);
        build_points(L, d);
      }
      continue;
    }
    const int s = __builtin_amdgcn_readfirstlane(sg);
    if (dn != d || s < 0 || s >= job.nseg || npoints(d) > job.pe) { err = TRK_E_INTERNAL; break; }
    uint32_t* acc = job.segacc + (size_t)s * job.pe;
    const int P = npoints(d);
    if (op == DG_S || op == DG_SDG || op == DG_Z || op == DG_CZ) {
      for (int p = lane; p < P; p += TL) {
        uint32_t Y = L.Ys[p];
        int ba = getb(L.hbN[0], a), bb = op == DG_CZ ? getb(L.hbN[0], b) : 0;
        while (Y) {
          const int j = __builtin_ctz(Y);
          Y &= Y - 1;
          ba ^= getb(L.hbN[1 + j], a);
          if (op == DG_CZ) bb ^= getb(L.hbN[1 + j], b);
        }
        const int mu = op == DG_S ? ba : op == DG_SDG ? 3 * ba : op == DG_Z ? 2 * ba : 2 * (ba & bb);
        __hip_atomic_fetch_add(gmem(&acc[p]), (uint32_t)(mu & 3), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      // (the index, b* basis and images stay; the rows and signs change)
      cur = nx;
      continue;
    }
    ph_save_old(L, cur, pr, n, d);
    const int kold = pr.k;
    cur = nx;
    ph_load(L, cur, pr, n, d);
    const int knew = pr.k;
    const int dk = knew - kold;
    const bool hsplit = op == DG_H && dk == 0;
    for (int p = lane; p < P; p += TL) {
      uint32_t Y = L.Ys[p];
      uint64_t so[SF_WMAX], bo[SF_WMAX], bn[SF_WMAX], src[SF_WMAX];
      point_vec(L.os0, L.oV, Y, 0, so);
      point_vec(L.hbO[0], L.hbO, Y, 1, bo);
      point_vec(L.hbN[0], L.hbN, Y, 1, bn);
      int e = 0, t = 0;
      int ba = getb(bn, a);
      for (int w = 0; w < W; ++w) src[w] = bn[w];
      if (op != DG_H) {
        int mu = 0;
        switch (op) {
          case DG_X: flipb(src, a); break;
          case DG_Y: flipb(src, a); mu = ba ? 1 : 3; break;
          case DG_CNOT: if (ba) flipb(src, b); break;
        }
        int u = uexp(L, so, bo, src);
        if (u < 0) err = TRK_E_INTERNAL;
        e = mu + u;
      } else {
        uint64_t b1[SF_WMAX];
        for (int w = 0; w < W; ++w) b1[w] = bn[w];
        if (ba) flipb(src, a); else flipb(b1, a);   // src: bit a = 0, b1: bit a = 1
        if (dk == 1) {
          int u0 = uexp(L, so, bo, src);
          int u1 = uexp(L, so, bo, b1);
          if ((u0 < 0) == (u1 < 0)) err = TRK_E_INTERNAL;
          e = u0 >= 0 ? u0 : u1 + 2 * ba;
        } else if (dk == -1) {
          int u0 = uexp(L, so, bo, src);
          if (u0 < 0) err = TRK_E_INTERNAL;
          e = u0;
        } else {
          int e0 = uexp(L, so, bo, src);
          int e1 = uexp(L, so, bo, b1);
          if (e0 < 0 || e1 < 0) err = TRK_E_INTERNAL;
          e1 += 2 * ba;
          int dl = (e1 - e0) & 3;
          if (!(dl & 1)) err = TRK_E_INTERNAL;
          e = e0;
          t = dl == 3 ? 1 : 0;        // omega = exp(i pi (2 e0 + 1 - 2t)/4)
        }
      }
      __hip_atomic_fetch_add(gmem(&acc[p]), (uint32_t)(e & 3), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (hsplit) L.t0[p] = (uint8_t)t;
    }
    __syncthreads();
    const int hi = __builtin_amdgcn_readfirstlane(hg);
    if (hsplit != (hi >= 0)) err = TRK_E_INTERNAL;
    else if (hsplit) fit_gf2(L, L.t0, d, &job.had[hi]);
    __syncthreads();
    err = wave_max(err);
  }
  err = wave_max(err);
  if (err && lane == 0) st->error = err;
}

static __device__ void track_body(LL& L, const TrackJob& job) {
  TrackState* st = job.st;
  const int lane = lane_id();
  // (sizes and gate fields are the same in every lane: read as scalars so
  // that the gate dispatch and the bit positions stay scalar)
  const int n = __builtin_amdgcn_readfirstlane(st->n);
  int d = __builtin_amdgcn_readfirstlane(st->d);
  int err = 0;
  if (lane_id() < 16) L.tc[lane_id()] = 0;
  for (int i = lane; i < 2 * LL::RN; i += TL) L.lst[i] = 0u;
  if (lane == 0) L.misc[1] = 0;
  __syncthreads();
  TIC(7);
  // load state
  for (int i = lane; i < LL::RN * LL::RW; i += TL) {
    const int r = i / LL::RW, w = i % LL::RW;  // TrackState rows hold SF_WMAX words
    L.rx[i] = r < n ? st->rx[r * SF_WMAX + w] : 0ull;
    L.rz[i] = r < n ? st->rz[r * SF_WMAX + w] : 0ull;
    L.cx[i] = r < n ? st->cx[r * SF_WMAX + w] : 0ull;
    L.cz[i] = r < n ? st->cz[r * SF_WMAX + w] : 0ull;
  }
  if (lane < SF_WMAX) L.s0[lane] = st->s0[lane];
  if (lane < d) for (int w = 0; w < SF_WMAX; ++w) L.V[lane][w] = st->V[lane][w];
  __syncthreads();
  // deferred filter of the last measurement (needs its outcome)
  if (st->pend) apply_pending(L, st, job.dry ? nullptr : job.outcomes, &d);
  if (!job.dry) build_points(L, d);
  __syncthreads();
  Regs TB;
  regs_load(L, TB, n);
  // the Clifford loop needs only each row's lead (terminal steps rebuild the
  // pivot index from the rows)
  for (int k = 0; k < W; ++k) TB.ld[k] = 64 * k + lane < n ? row_lead_sel(TB.x[k], TB.z[k], n) : -1;
  // this kernel conjugates, repairs and records; the phase kernels evaluate
  // the Clifford gates' phases from the records
  const bool rec = !job.dry;
  if (rec && !job.rec) {
    if (lane == 0 && !st->error) st->error = TRK_E_INTERNAL;
    return;
  }
  // the Clifford loop keeps the hull and the lead-stamp generation in
  // registers; terminal steps work on the LDS copies
  uint64_t HB[W];
  hull_to_regs(L, HB, d);
  uint32_t gen = (uint32_t)L.misc[1];
  int kx = count_x(TB, n);
  if (rec) {
    rec_write(job, 0, TB, HB, n, d);
    seg_clear(job, 0, d);
  }
  int seg = 0, nhad = 0, had_base = 0, nmeas = st->nmeas, dmax = st->dmax;
  int pend = 0, pend_j0 = -1, pend_c0 = 0, pend_meas = -1;
  uint32_t pend_r = 0;
  bool open = false;
  // errors of Clifford steps are per lane until the next terminal step or
  // the end of the range; errw is the wave-uniform copy that stops the loop
  int errw = 0;
  DGate nxt;
  memset(&nxt, 0, sizeof nxt);
  if (job.g0 < job.g1) nxt = load_gate(job.gates + job.g0);
  for (int g = job.g0; g < job.g1 && !errw; ++g) {
    DGate gt = nxt;
    gt.op = __builtin_amdgcn_readfirstlane(gt.op);
    gt.q0 = __builtin_amdgcn_readfirstlane(gt.q0);
    gt.q1 = __builtin_amdgcn_readfirstlane(gt.q1);
    gt.q2 = __builtin_amdgcn_readfirstlane(gt.q2);
    if (g + 1 < job.g1) nxt = load_gate(job.gates + g + 1);  // next gate's load overlaps this one
    const int gi = g - job.g0;
    if (gt.op < DG_NCPHASE) {
      const bool hs = clifford_gate_rec(L, TB, HB, gen, gt.op, gt.q0, gt.q1, n, d, &kx);
      if (rec) {
        TIC(0);
        if (lane == 0) {
          *gmem(job.ginfo + 2 * gi) = seg;
          *gmem(job.ginfo + 2 * gi + 1) = hs ? had_base + nhad : -1;
        }
        rec_write(job, gi + 1, TB, HB, n, d);
        TOC(0);
      }
      if (hs) ++nhad;
      open = true;
      continue;
    }
    TIC(6);
    // the load-time dry run records the hull dimension on entry to every
    // terminal gate (the sizes of the element launches)
    if (job.dry && job.ginfo && lane == 0) *gmem(job.ginfo + gi) = d;
    // terminal gate of the segment: works on the LDS copy of the tableau
    regs_store(L, TB, n, true);
    hull_to_lds(L, HB, d);
    if (lane == 0) L.misc[1] = (int)gen;
    __syncthreads();
    // the Clifford steps keep no pivot index, b* basis or hull images
    rebuild_index(L, n);
    if (rec) {
      build_beta(L, n);
      hull_images(L, L.hbN, d, false);
      if (lane == 0) { *gmem(job.ginfo + 2 * gi) = -1; *gmem(job.ginfo + 2 * gi + 1) = -1; }
    }
    if (gt.op == DG_CPH2 || gt.op == DG_CX2) {
      terminal_controlled(L, job, gt, seg, nhad, had_base, n, &d, &err);
      if (d > dmax) dmax = d;
      if (d > SF_DMAX - 1) err = TRK_E_DIM;
      err = wave_max(err);
      errw = err;
      __syncthreads();
      regs_load(L, TB, n);
      hull_to_regs(L, HB, d);
      gen = (uint32_t)L.misc[1];
      kx = count_x(TB, n);
      if (rec) {
        rec_write(job, gi + 1, TB, HB, n, d);
        seg_clear(job, seg + 1, d);
      }
      TOC(6);
      had_base += nhad;
      nhad = 0;
      ++seg;
      open = false;
      if (!job.dry) build_points(L, d);
      __syncthreads();
      continue;
    }
    const int q = gt.q0;
    const bool is_meas = gt.op == DG_MEASURE;
    SegProg* sp = job.dry ? nullptr : job.prog + seg;
    const int R = (n + 63) / 64;
    int rnd = 0;
    for (int it = 0; it < R; ++it) {
      int i = it * 64 + lane;
      rnd |= __ballot(i < n && getb(&L.rx[i * LL::RW], q)) != 0ull;
    }
    int d_entry = d;
    if (!job.dry) {
      if (lane == 0) emit_header(sp, SEG_NONE, is_meas, d, d, nhad, had_base);
      zero_z4(&sp->E);
      __syncthreads();
    }
    if (!rnd) {
      uint32_t c0, r;
      det_functional(L, q, n, d, &c0, &r, &err);
      if (!job.dry && lane == 0) {
        if (is_meas) { sp->m_c0 = c0; sp->m_r = r; sp->m_j0 = r ? 31 - __builtin_clz(r) : -1; }
        else { sp->kind = SEG_DET; sp->det_c = c0; sp->det_r = r; sp->ph_re = gt.c; sp->ph_im = gt.s; }
      }
      if (!job.dry) { zero_z4(&sp->B0); zero_z4(&sp->B1); }
      if (is_meas) {
        pend = 1; pend_r = r; pend_c0 = (int)c0; pend_j0 = r ? 31 - __builtin_clz(r) : -1;
        pend_meas = nmeas;
        if (!job.dry && lane == 0) sp->meas_index = nmeas;
        nmeas++;
      }
    } else {
      save_old(L, n, d);
      // d_q: rows anticommuting with Z_q; pivot p = the one with the largest lead
      if (lane < SF_WMAX) L.dq[lane] = 0;
      __syncthreads();
      int p = -1, pl = -1;
      for (int it = 0; it < R; ++it) {
        int i = it * 64 + lane;
        bool has = i < n && getb(&L.rx[i * LL::RW], q);
        uint64_t bb = __ballot(has);
        if (lane == 0) L.dq[it] = bb;
        int myl = has ? (int)L.lead[i] : -1;
        for (int o = 32; o > 0; o >>= 1) {
          int ol = __shfl_xor(myl, o);
          myl = ol > myl ? ol : myl;
        }
        if (myl > pl) {
          pl = myl;
          uint64_t bw = __ballot(has && L.lead[i] == myl);
          p = it * 64 + __builtin_ctzll(bw);
        }
      }
      __syncthreads();
      // rows i != p with X/Y at q: row_i <- row_i * row_p
      if (lane == 0) for (int w = 0; w < SF_WMAX; ++w) { L.rmask[w] = 0; L.cmask[w] = 0; }
      __syncthreads();
      for (int it = 0; it < R; ++it) {
        int i = it * 64 + lane;
        if (i >= n || i == p || !getb(&L.dq[0], i)) continue;
        int c = rowprod_sign(&L.rx[i * LL::RW], &L.rz[i * LL::RW], &L.rx[p * LL::RW], &L.rz[p * LL::RW]);
        for (int w = 0; w < W; ++w) { L.rx[i * LL::RW + w] ^= L.rx[p * LL::RW + w]; L.rz[i * LL::RW + w] ^= L.rz[p * LL::RW + w]; }
        atomicOr((unsigned long long*)&L.rmask[i >> 6], 1ull << (i & 63));
        if (c) atomicOr((unsigned long long*)&L.cmask[i >> 6], 1ull << (i & 63));
      }
      __syncthreads();
      cols_rowsum(L, p, n);
      apply_rowsum_batch(L, p, d, false);
      // row p := Z_q with sign x; child x of each element sets phase bit p to x
      for (int it = 0; it < R; ++it) {
        const int qq = it * 64 + lane;
        if (qq < n) {
          L.cx[qq * LL::RW + (p >> 6)] &= ~(1ull << (p & 63));
          L.cz[qq * LL::RW + (p >> 6)] &= ~(1ull << (p & 63));
        }
      }
      __syncthreads();
      if (lane == 0) {
        for (int w = 0; w < W; ++w) { L.rx[p * LL::RW + w] = 0; L.rz[p * LL::RW + w] = 0; }
        for (int w = 0; w < SF_WMAX; ++w) L.u[w] = 0;
        flipb(&L.rz[p * LL::RW], q);
        flipb(&L.cz[q * LL::RW], p);
        flipb(L.u, p);
        if (getb(L.s0, p)) flipb(L.s0, p);
      }
      __syncthreads();
      if (lane < d && getb(L.V[lane], p)) flipb(L.V[lane], p);
      for (int it = 0; it < R; ++it) {
        int i = it * 64 + lane;
        if (i >= n) continue;
        L.lead[i] = (int16_t)row_lead(&L.rx[i * LL::RW], &L.rz[i * LL::RW], n);
      }
      __syncthreads();
      repair(L, n, d, true, 0);
      rebuild_index(L, n);
      const uint32_t delta = span_reduce(L.oV, L.dq, d, nullptr, nullptr);
      if (!job.dry) {
        build_beta(L, n);
        hull_images(L, L.hbN, d, true);
        // cofactor amplitude factors beta_x(Y) (sampled, fitted)
        const int P = npoints(d);
        for (int pt = lane; pt < P; pt += TL) {
          uint32_t Y = L.Ys[pt];
          uint64_t so[SF_WMAX], bo[SF_WMAX], bc[SF_WMAX];
          point_vec(L.os0, L.oV, Y, 0, so);
          point_vec(L.hbO[0], L.hbO, Y, 1, bo);
          point_vec(L.hbN[0], L.hbN, Y, 1, bc);
          int e0 = uexp(L, so, bo, bc);
          for (int w = 0; w < W; ++w) bc[w] ^= L.hbN[d + 1][w];
          int e1 = uexp(L, so, bo, bc);
          if (e0 < 0 || e1 < 0) err = TRK_E_INTERNAL;
          L.t0[pt] = (uint8_t)(e0 & 3);
          L.t1[pt] = (uint8_t)(e1 & 3);
        }
        __syncthreads();
        fit_z4(L, L.t0, d, &sp->B0, &err);
        fit_z4(L, L.t1, d, &sp->B1, &err);
        __syncthreads();
      }
      // hull after the split
      int kind;
      if (delta == 0xffffffffu) {
        kind = SEG_GROW;
        if (lane == 0) for (int w = 0; w < SF_WMAX; ++w) L.V[d][w] = L.u[w];
        __syncthreads();
        d += 1;
      } else {
        kind = SEG_PAIR;
        int j0 = 31 - __builtin_clz(delta);
        if (lane == 0) {
          uint64_t v[SF_WMAX], hbv[SF_WMAX];
          for (int w = 0; w < SF_WMAX; ++w) { v[w] = L.u[w]; hbv[w] = L.hbN[d + 1][w]; }
          for (int j = 0; j < d; ++j)
            if (j != j0 && ((delta >> j) & 1u))
              for (int w = 0; w < SF_WMAX; ++w) { v[w] ^= L.V[j][w]; hbv[w] ^= L.hbN[1 + j][w]; }
          for (int w = 0; w < SF_WMAX; ++w) { L.V[j0][w] = v[w]; L.hbN[1 + j0][w] = hbv[w]; }
        }
        __syncthreads();
        if (!job.dry && lane == 0) { sp->j0 = j0; sp->delta = delta; }
      }
      if (!job.dry && lane == 0) {
        sp->kind = kind; sp->d_out = d;
        if (!is_meas) { sp->ph_re = gt.c; sp->ph_im = gt.s; }
      }
      // the dry run marks measurements whose cofactor grows the hull (their
      // segment pass is folded into the measurement kernels; the kind does
      // not depend on outcomes)
      if (job.dry && job.ginfo && lane == 0 && is_meas && kind == SEG_GROW)
        *gmem(job.ginfo + gi) = d_entry | SF_DTRACE_GROW;
      if (is_meas) {
        uint32_t c0, r;
        det_functional(L, q, n, d, &c0, &r, &err);
        pend = 1; pend_r = r; pend_c0 = (int)c0; pend_j0 = r ? 31 - __builtin_clz(r) : -1;
        pend_meas = nmeas;
        if (!job.dry && lane == 0) { sp->m_c0 = c0; sp->m_r = r; sp->m_j0 = pend_j0; sp->meas_index = nmeas; }
        nmeas++;
      }
    }
    if (d > dmax) dmax = d;
    if (d > SF_DMAX - 1) err = TRK_E_DIM;
    err = wave_max(err);
    errw = err;
    __syncthreads();
    regs_load(L, TB, n);
    hull_to_regs(L, HB, d);
    gen = (uint32_t)L.misc[1];
    kx = count_x(TB, n);
    if (rec) {
      rec_write(job, gi + 1, TB, HB, n, d);
      seg_clear(job, seg + 1, d);
    }
    TOC(6);
    // new segment
    had_base += nhad;
    nhad = 0;
    ++seg;
    open = false;
    if (is_meas) {
      if (job.dry) {
        // outcome-independent part of the filter: the dimension
        if (pend_r != 0) {
          uint64_t vj0[SF_WMAX];
          for (int w = 0; w < SF_WMAX; ++w) vj0[w] = L.V[pend_j0][w];
          __syncthreads();
          uint64_t mine[SF_WMAX];
          if (lane < d) for (int w = 0; w < SF_WMAX; ++w) mine[w] = L.V[lane][w] ^ (((pend_r >> lane) & 1u) ? vj0[w] : 0ull);
          __syncthreads();
          if (lane < d && lane != pend_j0) {
            int dst = lane < pend_j0 ? lane : lane - 1;
            for (int w = 0; w < SF_WMAX; ++w) L.V[dst][w] = mine[w];
          }
          d -= 1;
          __syncthreads();
        }
        pend = 0;
        hull_to_regs(L, HB, d);
      } else {
        // the range ends at a measurement (the host splits ranges there)
        break;
      }
    }
    if (!job.dry) build_points(L, d);
    __syncthreads();
  }
  err = wave_max(err);
  if (open && !job.dry && !err) {
    SegProg* sp = job.prog + seg;
    if (lane == 0) emit_header(sp, SEG_NONE, 0, d, d, nhad, had_base);
    zero_z4(&sp->E);
    zero_z4(&sp->B0);
    zero_z4(&sp->B1);
    ++seg;
  }
  regs_store(L, TB, n, true);
  hull_to_lds(L, HB, d);
  __syncthreads();
  // write back
  for (int i = lane; i < n * LL::RW; i += TL) {
    const int r = i / LL::RW, w = i % LL::RW;
    st->rx[r * SF_WMAX + w] = L.rx[i];
    st->rz[r * SF_WMAX + w] = L.rz[i];
    st->cx[r * SF_WMAX + w] = L.cx[i];
    st->cz[r * SF_WMAX + w] = L.cz[i];
  }
  if (lane < SF_WMAX) st->s0[lane] = L.s0[lane];
  if (lane < d) for (int w = 0; w < SF_WMAX; ++w) st->V[lane][w] = L.V[lane][w];
  if (lane == 0) {
    st->d = d;
    st->nmeas = nmeas;
    st->pend = job.dry ? 0 : pend;
    st->pend_r = pend_r; st->pend_c0 = pend_c0; st->pend_j0 = pend_j0; st->pend_meas = pend_meas;
    st->dmax = dmax;
    if (err && !st->error) st->error = err;
    L.tc[7] += TCLOCK();
    for (int k = 0; k < 16; ++k) st->cycles[k] += L.tc[k];
  }
}
};

// LDS-resident variant of the tableau track (rows in LDS, elimination in
// registers per call), used for frames of more than 128 qubits: keeping the
// whole tableau in registers there spills to scratch.
template <int W>
struct TrkL {
static __device__ int row_lead(const uint64_t* x, const uint64_t* z, int n) {
  for (int w = 0; w < W; ++w) if (x[w]) return 64 * w + __builtin_ctzll(x[w]);
  for (int w = 0; w < W; ++w) if (z[w]) return n + 64 * w + __builtin_ctzll(z[w]);
  return -1;
}

// Sign bit c of row1 * row2 = (-1)^c (row1 xor row2) for commuting rows,
// from the literal products of Table 1 (XY=iZ, YZ=iX, ZX=iY; reversed -i).
static __device__ int rowprod_sign(const uint64_t* x1, const uint64_t* z1, const uint64_t* x2,
                            const uint64_t* z2) {
  int pos = 0, neg = 0;
  for (int w = 0; w < W; ++w) {
    uint64_t a = x1[w], b = z1[w], c = x2[w], d = z2[w];
    pos += __popcll((a & b & ~c & d) | (a & ~b & c & d) | (~a & b & c & ~d));
    neg += __popcll((a & b & c & ~d) | (a & ~b & ~c & d) | (~a & b & c & d));
  }
  return ((pos - neg) & 3) >> 1;
}

// ---------------------------------------------------------------------------
// Echelon bookkeeping
// ---------------------------------------------------------------------------
static __device__ void rebuild_index(Lds& L, int n) {
  const int lane = lane_id();
  for (int i = lane; i < SF_NMAX; i += TL) { L.xpiv[i] = -1; L.zpiv[i] = -1; }
  __syncthreads();
  for (int i = lane; i < n; i += TL) {
    int ld = row_lead(&L.rx[i * SF_WMAX], &L.rz[i * SF_WMAX], n);
    L.lead[i] = (int16_t)ld;
    if (ld >= 0 && ld < n) L.xpiv[ld] = (int16_t)i;
    else if (ld >= n) L.zpiv[ld - n] = (int16_t)i;
  }
  __syncthreads();
  const int R = (n + 63) / 64;
  int k = 0;
  for (int it = 0; it < R; ++it) {
    int i = it * 64 + lane;
    bool isx = i < n && L.lead[i] >= 0 && L.lead[i] < n;
    bool isz = i < n && L.lead[i] >= n;
    uint64_t bx = __ballot(isx), bz = __ballot(isz);
    k += __popcll(bx);
    if (lane == 0) L.zsm[it] = bz;
  }
  if (lane == 0) {
    for (int it = R; it < SF_WMAX; ++it) L.zsm[it] = 0;
    L.misc[0] = k;
  }
  __syncthreads();
}

// Tracked phase-vector images: s0 (affine), V[0..d) and optionally u (linear).
// Apply sigma_i ^= sigma_m ^ c_i for every i in rmask (c in cmask).
static __device__ void apply_rowsum_batch(Lds& L, int m, int d, bool with_u) {
  const int lane = lane_id();
  uint64_t* vec = nullptr;
  bool affine = false;
  if (lane < d) vec = L.V[lane];
  else if (lane == d) { vec = L.s0; affine = true; }
  else if (lane == d + 1 && with_u) vec = L.u;
  if (vec) {
    int bm = getb(vec, m);
    for (int w = 0; w < W; ++w) vec[w] ^= (bm ? L.rmask[w] : 0ull) ^ (affine ? L.cmask[w] : 0ull);
  }
  __syncthreads();
}

// Column-major copy of the tableau: L.cx[q] / L.cz[q] hold the slots whose
// row has an x (z) bit at qubit q.  The track kernels keep it in the state, in
// step with every row change; the readout builds it from the rows.
static __device__ void build_cols(Lds& L, int n) {
  const int lane = lane_id();
  // 64 x 64 blocks: rows 64 k.., columns 64 w..; after the transpose lane c
  // holds word k of column 64 w + c
  for (int k = 0; k < W; ++k) {
    const int i = 64 * k + lane;
    for (int w = 0; w < W; ++w) {
      const uint64_t tx = transpose64(i < n ? L.rx[i * SF_WMAX + w] : 0ull);
      const uint64_t tz = transpose64(i < n ? L.rz[i * SF_WMAX + w] : 0ull);
      const int q = 64 * w + lane;
      if (q < n) { L.cx[q * SF_WMAX + k] = tx; L.cz[q * SF_WMAX + k] = tz; }
    }
  }
  __syncthreads();
}

// rows in L.rmask received row m: toggle those slots in every column where
// row m has a bit
static __device__ void cols_rowsum(Lds& L, int m, int n) {
  const int lane = lane_id();
  const int R = (n + 63) / 64;
  for (int it = 0; it < R; ++it) {
    const int q = it * 64 + lane;
    if (q >= n) continue;
    if (getb(&L.rx[m * SF_WMAX], q))
      for (int w = 0; w < W; ++w) L.cx[q * SF_WMAX + w] ^= L.rmask[w];
    if (getb(&L.rz[m * SF_WMAX], q))
      for (int w = 0; w < W; ++w) L.cz[q * SF_WMAX + w] ^= L.rmask[w];
  }
}

// Gaussian elimination restricted to the columns that break the echelon
// form: a column breaks it when it is the lead of some row and at least two
// rows have a bit there (on z columns only Z-block rows count, unless full).
// full = 0 keeps the form of Figure 2b (X-block reduced on x-leads, Z-block
// reduced on z-leads); full = 1 also clears X-block bits on z-leads.  Each
// step takes the smallest such column, multiplies its first leading row into
// every other row with a bit there, and replays the row multiplication on the
// tracked phase vectors.
// Rows, their leads, the column-major copy and the tracked phase vectors are
// held in registers for the whole loop: lane l owns
// row slots and columns 64k + l (k < W) and hull vector l (V[l], then s0 at
// lane d, u at lane d + 1).  The pivot row travels by readlane, the row masks
// of each step by ballot; LDS is read on entry and written on exit only.
static __device__ void repair(Lds& L, int n, int d, bool with_u, int full) {
  const int lane = lane_id();
  uint64_t x[W][W], z[W][W], cxr[W][W], czr[W][W];
  int ld[W];
  bool valid[W];
  for (int k = 0; k < W; ++k) {
    const int i = 64 * k + lane;
    valid[k] = i < n;
    for (int w = 0; w < W; ++w) {
      x[k][w] = valid[k] ? L.rx[i * SF_WMAX + w] : 0ull;
      z[k][w] = valid[k] ? L.rz[i * SF_WMAX + w] : 0ull;
      cxr[k][w] = valid[k] ? L.cx[i * SF_WMAX + w] : 0ull;
      czr[k][w] = valid[k] ? L.cz[i * SF_WMAX + w] : 0ull;
    }
    ld[k] = valid[k] ? (int)L.lead[i] : -1;
  }
  const bool has_vec = lane < d || lane == d || (lane == d + 1 && with_u);
  const bool affine = lane == d;
  uint64_t hv[W];
  for (int w = 0; w < W; ++w)
    hv[w] = lane < d ? L.V[lane][w] : lane == d ? L.s0[w] : (lane == d + 1 && with_u) ? L.u[w] : 0ull;
  for (int guard = 0; guard < 4 * SF_NMAX + 8; ++guard) {
    TIC(8);
    // Z-block rows (no x bits)
    uint64_t zs[W];
    for (int k = 0; k < W; ++k) {
      uint64_t xa = 0;
      for (int w = 0; w < W; ++w) xa |= x[k][w];
      const uint64_t b = __ballot(valid[k] && xa == 0ull);
      zs[k] = full ? ~0ull : b;
    }
    // bit counts of my columns (z columns: Z-block rows only unless full)
    int cntx[W], cntz[W];
    for (int k = 0; k < W; ++k) {
      int a = 0, b = 0;
      for (int w = 0; w < W; ++w) { a += __popcll(cxr[k][w]); b += __popcll(czr[k][w] & zs[w]); }
      cntx[k] = a;
      cntz[k] = b;
    }
    // smallest lead column shared by two rows
    int best = 0x7fffffff;
    for (int k = 0; k < W; ++k) {
      const int c = ld[k];
      const bool isx = c >= 0 && c < n;
      const int cc = c < 0 ? 0 : (isx ? c : c - n);
      int cnt = 0;
      for (int kk = 0; kk < W; ++kk) {
        const int vx = __shfl(cntx[kk], cc & 63);
        const int vz = __shfl(cntz[kk], cc & 63);
        if ((cc >> 6) == kk) cnt = isx ? vx : vz;
      }
      if (c >= 0 && cnt >= 2 && c < best) best = c;
    }
    for (int o = 32; o > 0; o >>= 1) {
      const int t = __shfl_xor(best, o);
      best = t < best ? t : best;
    }
    TOC(8);
    if (best == 0x7fffffff) break;
    TIC(9);
    const int col = __builtin_amdgcn_readfirstlane(best);
    // pivot: the first slot leading at col
    int m = -1;
    for (int k = 0; k < W && m < 0; ++k) {
      const uint64_t b = __ballot(valid[k] && ld[k] == col);
      if (b) m = 64 * k + __builtin_ctzll(b);
    }
    const int km = m >> 6, lm = m & 63;
    uint64_t xm[W], zm[W];
    for (int w = 0; w < W; ++w) {
      uint64_t sx = 0, sz = 0;
      for (int kk = 0; kk < W; ++kk)
        if (kk == km) { sx = x[kk][w]; sz = z[kk][w]; }
      xm[w] = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(sx >> 32), lm) << 32) |
              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)sx, lm);
      zm[w] = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(sz >> 32), lm) << 32) |
              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)sz, lm);
    }
    const bool xcol = col < n;
    const int cb = xcol ? col : col - n;
    uint64_t rm[W], cm[W];
    for (int k = 0; k < W; ++k) {
      const int i = 64 * k + lane;
      uint64_t xa = 0, wsel = 0;
      for (int w = 0; w < W; ++w) {
        xa |= x[k][w];
        if ((cb >> 6) == w) wsel = xcol ? x[k][w] : z[k][w];
      }
      const bool hit = valid[k] && i != m && (xcol || full || xa == 0ull) && ((wsel >> (cb & 63)) & 1ull);
      int c = 0;
      if (hit) {
        c = rowprod_sign(x[k], z[k], xm, zm);
        for (int w = 0; w < W; ++w) { x[k][w] ^= xm[w]; z[k][w] ^= zm[w]; }
        ld[k] = row_lead(x[k], z[k], n);
      }
      rm[k] = __ballot(hit);
      cm[k] = __ballot(hit && c);
    }
    // the column-major copy: columns where row m has a bit get the hit rows
    for (int k = 0; k < W; ++k) {
      if (!valid[k]) continue;
      const bool bx = (xm[k] >> lane) & 1ull, bz = (zm[k] >> lane) & 1ull;
      for (int w = 0; w < W; ++w) {
        if (bx) cxr[k][w] ^= rm[w];
        if (bz) czr[k][w] ^= rm[w];
      }
    }
    TOC(9);
    TIC(10);
    // replay on the tracked phase vectors: sigma_i ^= sigma_m (^ c_i on s0)
    if (has_vec) {
      uint64_t wm = 0;
      for (int w = 0; w < W; ++w) if ((m >> 6) == w) wm = hv[w];
      const bool bm = (wm >> (m & 63)) & 1ull;
      for (int w = 0; w < W; ++w) hv[w] ^= (bm ? rm[w] : 0ull) ^ (affine ? cm[w] : 0ull);
    }
    TOC(10);
  }
  for (int k = 0; k < W; ++k) {
    const int i = 64 * k + lane;
    if (!valid[k]) continue;
    for (int w = 0; w < W; ++w) {
      L.rx[i * SF_WMAX + w] = x[k][w];
      L.rz[i * SF_WMAX + w] = z[k][w];
      L.cx[i * SF_WMAX + w] = cxr[k][w];
      L.cz[i * SF_WMAX + w] = czr[k][w];
    }
    L.lead[i] = (int16_t)ld[k];
  }
  if (lane < d) for (int w = 0; w < W; ++w) L.V[lane][w] = hv[w];
  else if (lane == d) for (int w = 0; w < W; ++w) L.s0[w] = hv[w];
  else if (lane == d + 1 && with_u) for (int w = 0; w < W; ++w) L.u[w] = hv[w];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// b*(sigma): smallest basis string of the support of psi(M, sigma).
// Flipping the sign of Z-block row h moves the support by e_{q_h} (X_{q_h}
// anticommutes with that row only); the result is then reduced on the X-block
// leads.  So b*(sigma) = XOR over Z-rows h with sigma_h = 1 of beta_h, with
// beta_h = e_{q_h} ^ (x-part of the X-row leading at q_h, if any).
// ---------------------------------------------------------------------------
static __device__ void build_beta(Lds& L, int n) {
  const int lane = lane_id();
  for (int h = lane; h < n; h += TL) {
    uint64_t* b = &L.beta[h * SF_WMAX];
    for (int w = 0; w < SF_WMAX; ++w) b[w] = 0;
    int ld = L.lead[h];
    if (ld >= n) {
      int q = ld - n;
      flipb(b, q);
      int l = L.xpiv[q];
      if (l >= 0)
        for (int w = 0; w < W; ++w) b[w] ^= L.rx[l * SF_WMAX + w];
    }
  }
  __syncthreads();
}

static __device__ void bimage(const Lds& L, const uint64_t* vec, uint64_t* out) {
  uint64_t acc[SF_WMAX] = {0, 0, 0, 0};
  for (int w = 0; w < W; ++w) {
    uint64_t bits = vec[w] & L.zsm[w];
    while (bits) {
      int h = 64 * w + __builtin_ctzll(bits);
      bits &= bits - 1;
      for (int v = 0; v < W; ++v) acc[v] ^= L.beta[h * SF_WMAX + v];
    }
  }
  for (int w = 0; w < W; ++w) out[w] = acc[w];
}

// images of s0 (index 0), V[j] (1+j) and, if with_u, u (index d+1) into hb
static __device__ void hull_images(Lds& L, uint64_t (*hb)[SF_WMAX], int d, bool with_u) {
  const int lane = lane_id();
  if (lane == 0) bimage(L, L.s0, hb[0]);
  else if (lane <= d) bimage(L, L.V[lane - 1], hb[lane]);
  else if (lane == d + 1 && with_u) bimage(L, L.u, hb[d + 1]);
  __syncthreads();
}

// exponent e with psi(M_old, sigma)(b) = 2^{-k/2} i^e, or -1 if b is outside
// the support.  psi ~ prod_l (I + g_l)/2 |b*>: the amplitude at b* ^ x_S is the
// phase of applying the X-block generators in S to |b*>.
static __device__ int uexp(const Lds& L, const uint64_t* sig, const uint64_t* bO, const uint64_t* b) {
  uint64_t v[SF_WMAX];
  for (int w = 0; w < W; ++w) v[w] = bO[w];
  int e = 0;
  for (int w = 0; w < W; ++w) {
    uint64_t D = (b[w] ^ bO[w]) & L.oxpm[w];
    while (D) {
      int q = 64 * w + __builtin_ctzll(D);
      D &= D - 1;
      int l = L.oxpiv[q];
      uint64_t zv = 0;
      for (int t = 0; t < W; ++t) zv ^= L.oz[l * SF_WMAX + t] & v[t];
      e += 2 * (getb(sig, l) ^ par64(zv)) + L.ow[l];
      for (int t = 0; t < W; ++t) v[t] ^= L.ox[l * SF_WMAX + t];
    }
  }
  for (int w = 0; w < W; ++w) if (v[w] != b[w]) return -1;
  return e & 3;
}

// ---------------------------------------------------------------------------
// Sample points and fitting of quadratic forms over the hull coordinates
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Save the pre-gate tableau and hull (needed by the phase evaluation)
// ---------------------------------------------------------------------------
static __device__ void save_old(Lds& L, int n, int d) {
  const int lane = lane_id();
  for (int i = lane; i < n; i += TL) {
    uint64_t wz = 0;
    for (int w = 0; w < SF_WMAX; ++w) {
      L.ox[i * SF_WMAX + w] = L.rx[i * SF_WMAX + w];
      L.oz[i * SF_WMAX + w] = L.rz[i * SF_WMAX + w];
    }
    int c = 0;
    for (int w = 0; w < W; ++w) c += __popcll(L.rx[i * SF_WMAX + w] & L.rz[i * SF_WMAX + w]);
    L.ow[i] = (uint8_t)(c & 3);
    L.oxpiv[i] = L.xpiv[i];
    (void)wz;
  }
  for (int i = n + lane; i < SF_NMAX; i += TL) L.oxpiv[i] = -1;
  if (lane < d) for (int w = 0; w < SF_WMAX; ++w) L.oV[lane][w] = L.V[lane][w];
  if (lane == d) for (int w = 0; w < SF_WMAX; ++w) L.os0[w] = L.s0[w];
  if (lane <= d + 1) for (int w = 0; w < SF_WMAX; ++w) L.hbO[lane][w] = L.hbN[lane][w];
  __syncthreads();
  for (int it = 0; it < SF_WMAX; ++it) {
    const int q = it * 64 + lane;
    const uint64_t m = __ballot(q < n && L.xpiv[q] >= 0);
    if (lane == 0) L.oxpm[it] = m;
  }
  __syncthreads();
}

// gather the (<= 2) hull vectors of point Y into sigma/b images
static __device__ __forceinline__ void point_vec(const uint64_t* base, const uint64_t (*vecs)[SF_WMAX], uint32_t Y,
                                          int off, uint64_t* out) {
  for (int w = 0; w < W; ++w) out[w] = base[w];
  while (Y) {
    int j = __builtin_ctz(Y);
    Y &= Y - 1;
    for (int w = 0; w < W; ++w) out[w] ^= vecs[j + off][w];
  }
}

// ---------------------------------------------------------------------------
// Clifford gate
// ---------------------------------------------------------------------------
// rec: split form (the phase kernel evaluates the phase factor; *hs_out tells
// whether this is a Hadamard that keeps the support size).
static __device__ void clifford_gate(Lds& L, int op, int a, int b, int n, int d, int dry, GF2Q* had_out,
                              int* nhad, int* err, bool rec, bool* hs_out) {
  const int lane = lane_id();
  const int R = (n + 63) / 64;
  *hs_out = false;
  if (op == DG_S || op == DG_SDG || op == DG_Z || op == DG_CZ) {
    // Diagonal gates change only z bits of X-block rows and flip only X-block
    // signs: the echelon form, the support and b*(sigma) stay as they are, and
    // U|b*> = mu(b*) |b*>, so omega(Y) = mu(b*(sigma(Y))).
    TIC(1);
    if (lane == 0)
      for (int w = 0; w < SF_WMAX; ++w) L.fmask[w] = 0;
    __syncthreads();
    for (int it = 0; it < R; ++it) {
      int i = it * 64 + lane;
      if (i >= n) continue;
      uint64_t* x = &L.rx[i * SF_WMAX];
      uint64_t* z = &L.rz[i * SF_WMAX];
      int xa = getb(x, a), za = getb(z, a), fl = 0;
      if (op == DG_S) { fl = xa & za; if (xa) flipb(z, a); }
      else if (op == DG_SDG) { fl = xa & (za ^ 1); if (xa) flipb(z, a); }
      else if (op == DG_Z) fl = xa;
      else {
        int xb = getb(x, b), zb = getb(z, b);
        fl = xa & xb & (za ^ zb);
        if (xb) flipb(z, a);
        if (xa) flipb(z, b);
      }
      if (fl) atomicOr((unsigned long long*)&L.fmask[i >> 6], 1ull << (i & 63));
    }
    if (lane < W) {
      const int w = lane;
      if (op == DG_S || op == DG_SDG) L.cz[a * SF_WMAX + w] ^= L.cx[a * SF_WMAX + w];
      else if (op == DG_CZ) {
        L.cz[a * SF_WMAX + w] ^= L.cx[b * SF_WMAX + w];
        L.cz[b * SF_WMAX + w] ^= L.cx[a * SF_WMAX + w];
      }
    }
    __syncthreads();
    if (lane < SF_WMAX) L.s0[lane] ^= L.fmask[lane];
    __syncthreads();
    TOC(1);
    if (dry || rec) return;
    TIC(4);
    const int P = npoints(d);
    for (int p = lane; p < P; p += TL) {
      uint32_t Y = L.Ys[p];
      int ba = getb(L.hbN[0], a), bb = op == DG_CZ ? getb(L.hbN[0], b) : 0;
      while (Y) {
        const int j = __builtin_ctz(Y);
        Y &= Y - 1;
        ba ^= getb(L.hbN[1 + j], a);
        if (op == DG_CZ) bb ^= getb(L.hbN[1 + j], b);
      }
      int mu = op == DG_S ? ba : op == DG_SDG ? 3 * ba : op == DG_Z ? 2 * ba : 2 * (ba & bb);
      L.acc[p] = (uint8_t)((L.acc[p] + mu) & 3);
    }
    __syncthreads();
    TOC(4);
    return;
  }
  TIC(0);
  if (!dry && !rec) save_old(L, n, d);
  TOC(0);
  const int kold = L.misc[0];
  if (lane == 0)
    for (int w = 0; w < SF_WMAX; ++w) L.fmask[w] = 0;
  __syncthreads();
  TIC(1);
  // column update (Table 2) and sign flips
  for (int it = 0; it < R; ++it) {
    int i = it * 64 + lane;
    if (i >= n) continue;
    uint64_t* x = &L.rx[i * SF_WMAX];
    uint64_t* z = &L.rz[i * SF_WMAX];
    int xa = getb(x, a), za = getb(z, a), fl = 0;
    switch (op) {
      case DG_H: fl = xa & za; if (xa != za) { flipb(x, a); flipb(z, a); } break;
      case DG_S: fl = xa & za; if (xa) flipb(z, a); break;
      case DG_SDG: fl = xa & (za ^ 1); if (xa) flipb(z, a); break;
      case DG_X: fl = za; break;
      case DG_Z: fl = xa; break;
      case DG_Y: fl = xa ^ za; break;
      case DG_CNOT: {
        int xb = getb(x, b), zb = getb(z, b);
        fl = xa & zb & (xb ^ za ^ 1);
        if (xa) flipb(x, b);
        if (zb) flipb(z, a);
        break;
      }
      case DG_CZ: {
        int xb = getb(x, b), zb = getb(z, b);
        fl = xa & xb & (za ^ zb);
        if (xb) flipb(z, a);
        if (xa) flipb(z, b);
        break;
      }
    }
    if (fl) atomicOr((unsigned long long*)&L.fmask[i >> 6], 1ull << (i & 63));
    L.lead[i] = (int16_t)row_lead(x, z, n);
  }
  // the same column operations on the column-major copy
  if (lane < W) {
    const int w = lane;
    uint64_t* cxa = &L.cx[a * SF_WMAX];
    uint64_t* cza = &L.cz[a * SF_WMAX];
    if (op == DG_H) {
      uint64_t t = cxa[w]; cxa[w] = cza[w]; cza[w] = t;
    } else if (op == DG_CNOT) {
      L.cx[b * SF_WMAX + w] ^= cxa[w];
      cza[w] ^= L.cz[b * SF_WMAX + w];
    }
  }
  __syncthreads();
  // sign flips broadcast to every phase vector: s0 ^= f
  if (lane < SF_WMAX) L.s0[lane] ^= L.fmask[lane];
  __syncthreads();
  TOC(1);
  TIC(2);
  repair(L, n, d, false, 0);
  TOC(2);
  TIC(3);
  rebuild_index(L, n);
  if (dry) { TOC(3); return; }
  const int knew = L.misc[0];
  if (rec) {
    *hs_out = op == DG_H && knew == kold;
    TOC(3);
    return;
  }
  build_beta(L, n);
  hull_images(L, L.hbN, d, false);
  TOC(3);
  // per-element phase factor omega(Y), sampled at the fitting points
  const int dk = knew - kold;
  const bool hsplit = op == DG_H && dk == 0;
  TIC(4);
  const int P = npoints(d);
  for (int p = lane; p < P; p += TL) {
    uint32_t Y = L.Ys[p];
    uint64_t so[SF_WMAX], bo[SF_WMAX], bn[SF_WMAX], src[SF_WMAX];
    point_vec(L.os0, L.oV, Y, 0, so);
    point_vec(L.hbO[0], L.hbO, Y, 1, bo);
    point_vec(L.hbN[0], L.hbN, Y, 1, bn);
    int e = 0, t = 0;
    int ba = getb(bn, a);
    for (int w = 0; w < W; ++w) src[w] = bn[w];
    if (op != DG_H) {
      int mu = 0;
      switch (op) {
        case DG_S: mu = ba; break;
        case DG_SDG: mu = (4 - ba) & 3; break;
        case DG_X: flipb(src, a); break;
        case DG_Z: mu = 2 * ba; break;
        case DG_Y: flipb(src, a); mu = ba ? 1 : 3; break;
        case DG_CNOT: if (ba) flipb(src, b); break;
        case DG_CZ: mu = 2 * (ba & getb(bn, b)); break;
      }
      int u = uexp(L, so, bo, src);
      if (u < 0) *err = TRK_E_INTERNAL;
      e = mu + u;
    } else {
      uint64_t b1[SF_WMAX];
      for (int w = 0; w < W; ++w) b1[w] = bn[w];
      if (ba) flipb(src, a); else flipb(b1, a);   // src: bit a = 0, b1: bit a = 1
      if (dk == 1) {
        int u0 = uexp(L, so, bo, src);
        int u1 = uexp(L, so, bo, b1);
        if ((u0 < 0) == (u1 < 0)) *err = TRK_E_INTERNAL;
        e = u0 >= 0 ? u0 : u1 + 2 * ba;
      } else if (dk == -1) {
        int u0 = uexp(L, so, bo, src);
        if (u0 < 0) *err = TRK_E_INTERNAL;
        e = u0;
      } else {
        int e0 = uexp(L, so, bo, src);
        int e1 = uexp(L, so, bo, b1);
        if (e0 < 0 || e1 < 0) *err = TRK_E_INTERNAL;
        e1 += 2 * ba;
        int dl = (e1 - e0) & 3;
        if (!(dl & 1)) *err = TRK_E_INTERNAL;
        e = e0;
        t = dl == 3 ? 1 : 0;        // omega = exp(i pi (2 e0 + 1 - 2t)/4)
      }
    }
    L.acc[p] = (uint8_t)((L.acc[p] + e) & 3);
    if (hsplit) L.t0[p] = (uint8_t)t;
  }
  __syncthreads();
  TOC(4);
  if (hsplit) {
    TIC(5);
    fit_gf2(L, L.t0, d, &had_out[*nhad]);
    *nhad += 1;
    __syncthreads();
    TOC(5);
  }
}

// ---------------------------------------------------------------------------
// span test: delta with XOR_{j in delta} oV[j] == dq (slot bit vectors), or
// 0xffffffff if dq is outside the span.  Single lane (d <= 30 vectors).
// ---------------------------------------------------------------------------
// Wave-parallel Gaussian elimination over the d vectors vecs[0..d) (one per
// lane).  Returns delta with XOR_{j in delta} vecs[j] == target, or
// 0xffffffff if the target is outside their span; tops[] receives the
// leading-bit positions of the echelon basis (in the order found).
static __device__ uint32_t span_reduce(const uint64_t (*vecs)[SF_WMAX], const uint64_t* target, int d,
                                       int* tops, int* ntops) {
  const int lane = lane_id();
  uint64_t v[W];
  uint32_t c = 0;
  const bool is_t = lane == 63;
  for (int w = 0; w < W; ++w) v[w] = lane < d ? vecs[lane][w] : (is_t && target ? target[w] : 0ull);
  if (lane < d) c = 1u << lane;
  bool used = false;
  int nt = 0;
  for (int round = 0; round < d; ++round) {
    uint64_t any = 0;
    for (int w = 0; w < W; ++w) any |= v[w];
    uint64_t bal = __ballot(lane < d && !used && any != 0ull);
    if (!bal) break;
    const int pl = __builtin_ctzll(bal);
    uint64_t pv[W];
    for (int w = 0; w < W; ++w) pv[w] = __shfl(v[w], pl);
    const uint32_t pc = __shfl(c, pl);
    int top = -1;
    for (int w = W - 1; w >= 0 && top < 0; --w) if (pv[w]) top = 64 * w + 63 - __builtin_clzll(pv[w]);
    if (tops && lane == 0) tops[nt] = top;
    ++nt;
    if (lane == pl) used = true;
    else if (getb(v, top)) {
      for (int w = 0; w < W; ++w) v[w] ^= pv[w];
      c ^= pc;
    }
  }
  if (ntops) *ntops = nt;
  uint64_t tany = 0;
  for (int w = 0; w < W; ++w) tany |= v[w];
  const uint64_t tz = __shfl(tany, 63);
  const uint32_t tc = __shfl(c, 63);
  return tz ? 0xffffffffu : tc;
}

// ---------------------------------------------------------------------------
// Non-Clifford phase gate or measurement on q: COFACTOR (section 3)
// ---------------------------------------------------------------------------
static __device__ void det_functional(Lds& L, int q, int n, int d, uint32_t* c0, uint32_t* r, int* err) {
  const int lane = lane_id();
  int h = L.zpiv[q];
  uint32_t rr = 0;
  if (h < 0) { if (lane == 0) *err = TRK_E_INTERNAL; h = 0; }
  else {
    for (int w = 0; w < W; ++w) {
      uint64_t want = (q >> 6) == w ? (1ull << (q & 63)) : 0ull;
      if (L.rz[h * SF_WMAX + w] != want || L.rx[h * SF_WMAX + w] != 0ull) *err = TRK_E_INTERNAL;
    }
  }
  rr = (uint32_t)__ballot(lane < d && getb(L.V[lane < d ? lane : 0], h));
  *c0 = (uint32_t)getb(L.s0, h);
  *r = rr;
}

// Filter step of a measurement on the hull: keep sigma(Y) with
// c0 ^ parity(r & Y) == outcome, i.e. fix coordinate j0 and drop it.

// ---------------------------------------------------------------------------
// Last step of a direct controlled phase / Toffoli (Eqs. 2 and 3): after the
// cofactors on the two controls both are deterministic, with values
// f1(Y) = c1 ^ parity(r1 & Y) and f2(Y) = c2 ^ parity(r2 & Y).  DG_CPH2 puts
// the phase on the elements with f1 & f2.  DG_CX2 applies X on q2 to them: X
// leaves the unsigned matrix as it is and flips the signs of the rows with a z
// bit at q2 (mask f), so such an element moves from sigma(Y) to sigma(Y) ^ f
// with the factor omega(Y) = psi(M, sigma(Y))(b*(sigma(Y) ^ f) ^ e_q2), a Z4
// quadratic form in Y (sampled and fitted as for the Clifford gates).  If f
// is in span(V) (f = sum of V[j], j in delta) the element moves to Y ^ delta,
// which has the same control values (f has no bit on the controls' Z rows);
// otherwise the hull grows by the coordinate V[d] = f.
// ---------------------------------------------------------------------------
static __device__ void terminal_controlled(Lds& L, const TrackJob& job, const DGate& gt, int seg, int nhad,
                                           int had_base, int n, int* dptr, int* err, bool rec) {
  const int lane = lane_id();
  int d = *dptr;
  SegProg* sp = job.dry ? nullptr : job.prog + seg;
  if (!job.dry) {
    if (lane == 0) emit_header(sp, SEG_DET2, 0, d, d, nhad, had_base);
    if (rec) zero_z4(&sp->E);   // fitted by the fit kernel when the range has Clifford gates
    else fit_z4(L, L.acc, d, &sp->E, err);
    __syncthreads();
  }
  uint32_t c1, r1, c2, r2;
  det_functional(L, gt.q0, n, d, &c1, &r1, err);
  det_functional(L, gt.q1, n, d, &c2, &r2, err);
  if (!job.dry && lane == 0) { sp->det_c = c1; sp->det_r = r1; sp->det2_c = c2; sp->det2_r = r2; }
  if (gt.op == DG_CPH2) {
    if (!job.dry) {
      if (lane == 0) { sp->kind = SEG_DET2; sp->ph_re = gt.c; sp->ph_im = gt.s; }
      zero_z4(&sp->B0);
      zero_z4(&sp->B1);
    }
    __syncthreads();
    return;
  }
  const int t = gt.q2;
  const int R = (n + 63) / 64;
  for (int it = 0; it < SF_WMAX; ++it) {
    const int i = it * 64 + lane;
    const uint64_t b = __ballot(it < R && i < n && getb(&L.rz[i * SF_WMAX], t));
    if (lane == 0) L.dq[it] = b;
  }
  __syncthreads();
  save_old(L, n, d);
  const uint32_t delta = span_reduce(L.oV, L.dq, d, nullptr, nullptr);
  if (!job.dry) {
    // b*(f): the images are linear, so b*(sigma(Y) ^ f) = b*(sigma(Y)) ^ b*(f)
    if (lane == 0) bimage(L, L.dq, L.hbN[d + 1]);
    __syncthreads();
    const int P = npoints(d);
    for (int pt = lane; pt < P; pt += TL) {
      const uint32_t Y = L.Ys[pt];
      uint64_t so[SF_WMAX], bo[SF_WMAX], src[SF_WMAX];
      point_vec(L.os0, L.oV, Y, 0, so);
      point_vec(L.hbO[0], L.hbO, Y, 1, bo);
      for (int w = 0; w < W; ++w) src[w] = bo[w] ^ L.hbN[d + 1][w];
      flipb(src, t);
      const int e = uexp(L, so, bo, src);
      if (e < 0) *err = TRK_E_INTERNAL;
      L.t0[pt] = (uint8_t)(e & 3);
    }
    __syncthreads();
    fit_z4(L, L.t0, d, &sp->B0, err);
    zero_z4(&sp->B1);
    __syncthreads();
  }
  if (delta != 0xffffffffu) {
    if (!job.dry && lane == 0) {
      sp->kind = SEG_CX2P;
      sp->delta = delta;
      sp->j0 = delta ? 31 - __builtin_clz(delta) : -1;
      sp->d_out = d;
    }
  } else {
    if (lane == 0)
      for (int w = 0; w < SF_WMAX; ++w) L.V[d][w] = L.dq[w];
    d += 1;
    if (!job.dry && lane == 0) { sp->kind = SEG_CX2G; sp->d_out = d; }
  }
  __syncthreads();
  *dptr = d;
}

// ---------------------------------------------------------------------------
// Split form for launches with few wide frames (as in Trk): records of the
// state after every gate from LDS, and the per-gate phase evaluation of the
// phase kernel.  Records hold W words per row part (LDS rows hold SF_WMAX).
// ---------------------------------------------------------------------------
static __device__ void rec_write(const TrackJob& job, int r, const Lds& L, int n, int d) {
  auto rw = gmem((uint64_t*)(job.rec + (size_t)r * job.rec_stride));
  const int lane = lane_id();
  for (int idx = lane; idx < n * W; idx += TL) {
    const int i = idx / W, w = idx % W;
    rw[i * 2 * W + w] = L.rx[i * SF_WMAX + w];
    rw[i * 2 * W + W + w] = L.rz[i * SF_WMAX + w];
  }
  auto hv = rw + (size_t)n * 2 * W;
  if (lane <= d)
    for (int w = 0; w < W; ++w) hv[lane * W + w] = lane == 0 ? L.s0[w] : L.V[lane - 1][w];
  if (lane == 0) *gmem((int32_t*)(job.rec + (size_t)r * job.rec_stride + ((size_t)n * 2 * W + (SF_DMAX + 1) * W) * 8)) = d;
}

static __device__ int rec_d(const TrackJob& job, int r, int n) {
  const uint64_t* rw = (const uint64_t*)(job.rec + (size_t)r * job.rec_stride);
  return *(const int32_t*)(rw + (size_t)n * 2 * W + (SF_DMAX + 1) * W);
}

static __device__ void rec_load(Lds& L, const TrackJob& job, int r, int n, int d) {
  auto rw = gmem((const uint64_t*)(job.rec + (size_t)r * job.rec_stride));
  const int lane = lane_id();
  for (int idx = lane; idx < SF_NMAX * SF_WMAX; idx += TL) {
    const int i = idx / SF_WMAX, w = idx % SF_WMAX;
    const bool in = i < n && w < W;
    L.rx[idx] = in ? rw[i * 2 * W + w] : 0ull;
    L.rz[idx] = in ? rw[i * 2 * W + W + w] : 0ull;
  }
  auto hv = rw + (size_t)n * 2 * W;
  if (lane <= d)
    for (int w = 0; w < SF_WMAX; ++w) {
      const uint64_t v = w < W ? hv[lane * W + w] : 0ull;
      if (lane == 0) L.s0[w] = v;
      else L.V[lane - 1][w] = v;
    }
  __syncthreads();
}

static __device__ void seg_clear(const TrackJob& job, int s, int d) {
  if (s >= job.nseg) return;
  const int P = min(npoints(d), job.pe);
  for (int p = lane_id(); p < P; p += TL) *gmem(job.segacc + (size_t)s * job.pe + p) = 0u;
}

// Phase factor of Clifford gate g0 + i from the records before and after it,
// added into its segment's sums (the evaluation of clifford_gate).
static __device__ void phase_gate(Lds& L, const TrackJob& job, int i) {
  const int lane = lane_id();
  const DGate gt = load_gate(job.gates + job.g0 + i);
  const int op = __builtin_amdgcn_readfirstlane(gt.op);
  if (op >= DG_NCPHASE) return;
  TrackState* st = job.st;
  const int n = __builtin_amdgcn_readfirstlane(st->n);
  const int d = __builtin_amdgcn_readfirstlane(rec_d(job, i + 1, n));
  const int s = __builtin_amdgcn_readfirstlane(*gmem(job.ginfo + 2 * i));
  if (d < 0 || d >= SF_DMAX || s < 0 || s >= job.nseg || npoints(d) > job.pe ||
      __builtin_amdgcn_readfirstlane(rec_d(job, i, n)) != d) {
    if (lane == 0) st->error = TRK_E_INTERNAL;
    return;
  }
  uint32_t* acc = job.segacc + (size_t)s * job.pe;
  const int a = __builtin_amdgcn_readfirstlane(gt.q0), b = __builtin_amdgcn_readfirstlane(gt.q1);
  int err = 0;
  const int P = npoints(d);
  if (op == DG_S || op == DG_SDG || op == DG_Z || op == DG_CZ) {
    rec_load(L, job, i + 1, n, d);
    rebuild_index(L, n);
    build_beta(L, n);
    hull_images(L, L.hbN, d, false);
    build_points(L, d);
    for (int p = lane; p < P; p += TL) {
      uint32_t Y = L.Ys[p];
      int ba = getb(L.hbN[0], a), bb = op == DG_CZ ? getb(L.hbN[0], b) : 0;
      while (Y) {
        const int j = __builtin_ctz(Y);
        Y &= Y - 1;
        ba ^= getb(L.hbN[1 + j], a);
        if (op == DG_CZ) bb ^= getb(L.hbN[1 + j], b);
      }
      const int mu = op == DG_S ? ba : op == DG_SDG ? 3 * ba : op == DG_Z ? 2 * ba : 2 * (ba & bb);
      __hip_atomic_fetch_add(gmem(&acc[p]), (uint32_t)(mu & 3), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  rec_load(L, job, i, n, d);
  rebuild_index(L, n);
  build_beta(L, n);
  hull_images(L, L.hbN, d, false);
  save_old(L, n, d);
  const int kold = L.misc[0];
  rec_load(L, job, i + 1, n, d);
  rebuild_index(L, n);
  build_beta(L, n);
  hull_images(L, L.hbN, d, false);
  const int knew = L.misc[0];
  build_points(L, d);
  const int dk = knew - kold;
  const bool hsplit = op == DG_H && dk == 0;
  for (int p = lane; p < P; p += TL) {
    uint32_t Y = L.Ys[p];
    uint64_t so[SF_WMAX], bo[SF_WMAX], bn[SF_WMAX], src[SF_WMAX];
    point_vec(L.os0, L.oV, Y, 0, so);
    point_vec(L.hbO[0], L.hbO, Y, 1, bo);
    point_vec(L.hbN[0], L.hbN, Y, 1, bn);
    int e = 0, t = 0;
    int ba = getb(bn, a);
    for (int w = 0; w < W; ++w) src[w] = bn[w];
    if (op != DG_H) {
      int mu = 0;
      switch (op) {
        case DG_X: flipb(src, a); break;
        case DG_Y: flipb(src, a); mu = ba ? 1 : 3; break;
        case DG_CNOT: if (ba) flipb(src, b); break;
      }
      int u = uexp(L, so, bo, src);
      if (u < 0) err = TRK_E_INTERNAL;
      e = mu + u;
    } else {
      uint64_t b1[SF_WMAX];
      for (int w = 0; w < W; ++w) b1[w] = bn[w];
      if (ba) flipb(src, a); else flipb(b1, a);   // src: bit a = 0, b1: bit a = 1
      if (dk == 1) {
        int u0 = uexp(L, so, bo, src);
        int u1 = uexp(L, so, bo, b1);
        if ((u0 < 0) == (u1 < 0)) err = TRK_E_INTERNAL;
        e = u0 >= 0 ? u0 : u1 + 2 * ba;
      } else if (dk == -1) {
        int u0 = uexp(L, so, bo, src);
        if (u0 < 0) err = TRK_E_INTERNAL;
        e = u0;
      } else {
        int e0 = uexp(L, so, bo, src);
        int e1 = uexp(L, so, bo, b1);
        if (e0 < 0 || e1 < 0) err = TRK_E_INTERNAL;
        e1 += 2 * ba;
        int dl = (e1 - e0) & 3;
        if (!(dl & 1)) err = TRK_E_INTERNAL;
        e = e0;
        t = dl == 3 ? 1 : 0;        // omega = exp(i pi (2 e0 + 1 - 2t)/4)
      }
    }
    __hip_atomic_fetch_add(gmem(&acc[p]), (uint32_t)(e & 3), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (hsplit) L.t0[p] = (uint8_t)t;
  }
  __syncthreads();
  const int hi = __builtin_amdgcn_readfirstlane(*gmem(job.ginfo + 2 * i + 1));
  if (hsplit != (hi >= 0)) err = TRK_E_INTERNAL;
  else if (hsplit) fit_gf2(L, L.t0, d, &job.had[hi]);
  __syncthreads();
  err = wave_max(err);
  if (err && lane == 0) st->error = err;
}

// chunk c of pchunk gates, one gate at a time
static __device__ void phase_body(Lds& L, const TrackJob& job, int c) {
  const int len = job.g1 - job.g0;
  const int k = job.pchunk > 0 ? job.pchunk : 1;
  const int i1 = min(len, (c + 1) * k);
  for (int i = c * k; i < i1; ++i) phase_gate(L, job, i);
}

static __device__ void track_body(Lds& L, const TrackJob& job) {
  TrackState* st = job.st;
  const int lane = lane_id();
  const int n = st->n;
  int d = st->d;
  int err = 0;
  if (lane_id() < 12) L.tc[lane_id()] = 0;
  __syncthreads();
  TIC(7);
  // load state
  for (int i = lane; i < SF_NMAX * SF_WMAX; i += TL) {
    L.rx[i] = i < n * SF_WMAX ? st->rx[i] : 0ull;
    L.rz[i] = i < n * SF_WMAX ? st->rz[i] : 0ull;
    L.cx[i] = i < n * SF_WMAX ? st->cx[i] : 0ull;
    L.cz[i] = i < n * SF_WMAX ? st->cz[i] : 0ull;
  }
  if (lane < SF_WMAX) L.s0[lane] = st->s0[lane];
  if (lane < d) for (int w = 0; w < SF_WMAX; ++w) L.V[lane][w] = st->V[lane][w];
  __syncthreads();
  // deferred filter of the last measurement (needs its outcome)
  if (st->pend) apply_pending(L, st, job.dry ? nullptr : job.outcomes, &d);
  rebuild_index(L, n);
  if (!job.dry) {
    build_beta(L, n);
    hull_images(L, L.hbN, d, false);
    build_points(L, d);
  }
  for (int p = lane; p < SF_PMAX; p += TL) L.acc[p] = 0;
  __syncthreads();
  // split form (when the job brings records): this kernel records, the phase
  // kernels evaluate
  const bool rec = !job.dry && job.rec != nullptr;
  if (rec) {
    rec_write(job, 0, L, n, d);
    seg_clear(job, 0, d);
  }
  int seg = 0, nhad = 0, had_base = 0, nmeas = st->nmeas, dmax = st->dmax;
  int pend = 0, pend_j0 = -1, pend_c0 = 0, pend_meas = -1;
  uint32_t pend_r = 0;
  bool open = false;
  DGate nxt;
  memset(&nxt, 0, sizeof nxt);
  if (job.g0 < job.g1) nxt = load_gate(job.gates + job.g0);
  for (int g = job.g0; g < job.g1 && !err; ++g) {
    const DGate gt = nxt;
    if (g + 1 < job.g1) nxt = load_gate(job.gates + g + 1);  // next gate's load overlaps this one
    const int gi = g - job.g0;
    if (gt.op < DG_NCPHASE) {
      bool hs = false;
      clifford_gate(L, gt.op, gt.q0, gt.q1, n, d, job.dry, job.had + had_base, &nhad, &err, rec, &hs);
      err = wave_max(err);
      if (rec) {
        if (lane == 0) {
          *gmem(job.ginfo + 2 * gi) = seg;
          *gmem(job.ginfo + 2 * gi + 1) = hs ? had_base + nhad : -1;
        }
        if (hs) ++nhad;
        rec_write(job, gi + 1, L, n, d);
      }
      open = true;
      continue;
    }
    TIC(6);
    if (job.dry && job.ginfo && lane == 0) *gmem(job.ginfo + gi) = d;
    if (rec) {
      // the Clifford steps of the split form keep no b* basis or images
      build_beta(L, n);
      hull_images(L, L.hbN, d, false);
      if (lane == 0) { *gmem(job.ginfo + 2 * gi) = -1; *gmem(job.ginfo + 2 * gi + 1) = -1; }
    }
    // terminal gate of the segment
    if (gt.op == DG_CPH2 || gt.op == DG_CX2) {
      terminal_controlled(L, job, gt, seg, nhad, had_base, n, &d, &err, rec);
      if (d > dmax) dmax = d;
      if (d > SF_DMAX - 1) err = TRK_E_DIM;
      err = wave_max(err);
      __syncthreads();
      if (rec) {
        rec_write(job, gi + 1, L, n, d);
        seg_clear(job, seg + 1, d);
      }
      TOC(6);
      had_base += nhad;
      nhad = 0;
      ++seg;
      open = false;
      if (!job.dry) {
        for (int pt = lane; pt < SF_PMAX; pt += TL) L.acc[pt] = 0;
        build_points(L, d);
      }
      __syncthreads();
      continue;
    }
    const int q = gt.q0;
    const bool is_meas = gt.op == DG_MEASURE;
    SegProg* sp = job.dry ? nullptr : job.prog + seg;
    const int R = (n + 63) / 64;
    int rnd = 0;
    for (int it = 0; it < R; ++it) {
      int i = it * 64 + lane;
      rnd |= __ballot(i < n && getb(&L.rx[i * SF_WMAX], q)) != 0ull;
    }
    int d_entry = d;
    if (!job.dry) {
      if (lane == 0) emit_header(sp, SEG_NONE, is_meas, d, d, nhad, had_base);
      if (rec) zero_z4(&sp->E);
      else fit_z4(L, L.acc, d, &sp->E, &err);
      __syncthreads();
    }
    if (!rnd) {
      uint32_t c0, r;
      det_functional(L, q, n, d, &c0, &r, &err);
      if (!job.dry && lane == 0) {
        if (is_meas) { sp->m_c0 = c0; sp->m_r = r; sp->m_j0 = r ? 31 - __builtin_clz(r) : -1; }
        else { sp->kind = SEG_DET; sp->det_c = c0; sp->det_r = r; sp->ph_re = gt.c; sp->ph_im = gt.s; }
      }
      if (!job.dry) { zero_z4(&sp->B0); zero_z4(&sp->B1); }
      if (is_meas) {
        pend = 1; pend_r = r; pend_c0 = (int)c0; pend_j0 = r ? 31 - __builtin_clz(r) : -1;
        pend_meas = nmeas;
        if (!job.dry && lane == 0) sp->meas_index = nmeas;
        nmeas++;
      }
    } else {
      save_old(L, n, d);
      // d_q: rows anticommuting with Z_q; pivot p = the one with the largest lead
      if (lane < SF_WMAX) L.dq[lane] = 0;
      __syncthreads();
      int p = -1, pl = -1;
      for (int it = 0; it < R; ++it) {
        int i = it * 64 + lane;
        bool has = i < n && getb(&L.rx[i * SF_WMAX], q);
        uint64_t bb = __ballot(has);
        if (lane == 0) L.dq[it] = bb;
        int myl = has ? (int)L.lead[i] : -1;
        for (int o = 32; o > 0; o >>= 1) {
          int ol = __shfl_xor(myl, o);
          myl = ol > myl ? ol : myl;
        }
        if (myl > pl) {
          pl = myl;
          uint64_t bw = __ballot(has && L.lead[i] == myl);
          p = it * 64 + __builtin_ctzll(bw);
        }
      }
      __syncthreads();
      // rows i != p with X/Y at q: row_i <- row_i * row_p
      if (lane == 0) for (int w = 0; w < SF_WMAX; ++w) { L.rmask[w] = 0; L.cmask[w] = 0; }
      __syncthreads();
      for (int it = 0; it < R; ++it) {
        int i = it * 64 + lane;
        if (i >= n || i == p || !getb(&L.dq[0], i)) continue;
        int c = rowprod_sign(&L.rx[i * SF_WMAX], &L.rz[i * SF_WMAX], &L.rx[p * SF_WMAX], &L.rz[p * SF_WMAX]);
        for (int w = 0; w < W; ++w) { L.rx[i * SF_WMAX + w] ^= L.rx[p * SF_WMAX + w]; L.rz[i * SF_WMAX + w] ^= L.rz[p * SF_WMAX + w]; }
        atomicOr((unsigned long long*)&L.rmask[i >> 6], 1ull << (i & 63));
        if (c) atomicOr((unsigned long long*)&L.cmask[i >> 6], 1ull << (i & 63));
      }
      __syncthreads();
      cols_rowsum(L, p, n);
      apply_rowsum_batch(L, p, d, false);
      // row p := Z_q with sign x; child x of each element sets phase bit p to x
      for (int it = 0; it < R; ++it) {
        const int qq = it * 64 + lane;
        if (qq < n) {
          L.cx[qq * SF_WMAX + (p >> 6)] &= ~(1ull << (p & 63));
          L.cz[qq * SF_WMAX + (p >> 6)] &= ~(1ull << (p & 63));
        }
      }
      __syncthreads();
      if (lane == 0) {
        for (int w = 0; w < SF_WMAX; ++w) { L.rx[p * SF_WMAX + w] = 0; L.rz[p * SF_WMAX + w] = 0; L.u[w] = 0; }
        flipb(&L.rz[p * SF_WMAX], q);
        flipb(&L.cz[q * SF_WMAX], p);
        flipb(L.u, p);
        if (getb(L.s0, p)) flipb(L.s0, p);
      }
      __syncthreads();
      if (lane < d && getb(L.V[lane], p)) flipb(L.V[lane], p);
      for (int it = 0; it < R; ++it) {
        int i = it * 64 + lane;
        if (i >= n) continue;
        L.lead[i] = (int16_t)row_lead(&L.rx[i * SF_WMAX], &L.rz[i * SF_WMAX], n);
      }
      __syncthreads();
      repair(L, n, d, true, 0);
      rebuild_index(L, n);
      const uint32_t delta = span_reduce(L.oV, L.dq, d, nullptr, nullptr);
      if (!job.dry) {
        build_beta(L, n);
        hull_images(L, L.hbN, d, true);
        // cofactor amplitude factors beta_x(Y) (sampled, fitted)
        const int P = npoints(d);
        for (int pt = lane; pt < P; pt += TL) {
          uint32_t Y = L.Ys[pt];
          uint64_t so[SF_WMAX], bo[SF_WMAX], bc[SF_WMAX];
          point_vec(L.os0, L.oV, Y, 0, so);
          point_vec(L.hbO[0], L.hbO, Y, 1, bo);
          point_vec(L.hbN[0], L.hbN, Y, 1, bc);
          int e0 = uexp(L, so, bo, bc);
          for (int w = 0; w < W; ++w) bc[w] ^= L.hbN[d + 1][w];
          int e1 = uexp(L, so, bo, bc);
          if (e0 < 0 || e1 < 0) err = TRK_E_INTERNAL;
          L.t0[pt] = (uint8_t)(e0 & 3);
          L.t1[pt] = (uint8_t)(e1 & 3);
        }
        __syncthreads();
        fit_z4(L, L.t0, d, &sp->B0, &err);
        fit_z4(L, L.t1, d, &sp->B1, &err);
        __syncthreads();
      }
      // hull after the split
      int kind;
      if (delta == 0xffffffffu) {
        kind = SEG_GROW;
        if (lane == 0) for (int w = 0; w < SF_WMAX; ++w) L.V[d][w] = L.u[w];
        __syncthreads();
        d += 1;
      } else {
        kind = SEG_PAIR;
        int j0 = 31 - __builtin_clz(delta);
        if (lane == 0) {
          uint64_t v[SF_WMAX], hbv[SF_WMAX];
          for (int w = 0; w < SF_WMAX; ++w) { v[w] = L.u[w]; hbv[w] = L.hbN[d + 1][w]; }
          for (int j = 0; j < d; ++j)
            if (j != j0 && ((delta >> j) & 1u))
              for (int w = 0; w < SF_WMAX; ++w) { v[w] ^= L.V[j][w]; hbv[w] ^= L.hbN[1 + j][w]; }
          for (int w = 0; w < SF_WMAX; ++w) { L.V[j0][w] = v[w]; L.hbN[1 + j0][w] = hbv[w]; }
        }
        __syncthreads();
        if (!job.dry && lane == 0) { sp->j0 = j0; sp->delta = delta; }
      }
      if (!job.dry && lane == 0) {
        sp->kind = kind; sp->d_out = d;
        if (!is_meas) { sp->ph_re = gt.c; sp->ph_im = gt.s; }
      }
      // the dry run marks measurements whose cofactor grows the hull (their
      // segment pass is folded into the measurement kernels; the kind does
      // not depend on outcomes)
      if (job.dry && job.ginfo && lane == 0 && is_meas && kind == SEG_GROW)
        *gmem(job.ginfo + gi) = d_entry | SF_DTRACE_GROW;
      if (is_meas) {
        uint32_t c0, r;
        det_functional(L, q, n, d, &c0, &r, &err);
        pend = 1; pend_r = r; pend_c0 = (int)c0; pend_j0 = r ? 31 - __builtin_clz(r) : -1;
        pend_meas = nmeas;
        if (!job.dry && lane == 0) { sp->m_c0 = c0; sp->m_r = r; sp->m_j0 = pend_j0; sp->meas_index = nmeas; }
        nmeas++;
      }
    }
    if (d > dmax) dmax = d;
    if (d > SF_DMAX - 1) err = TRK_E_DIM;
    err = wave_max(err);
    __syncthreads();
    if (rec) {
      rec_write(job, gi + 1, L, n, d);
      seg_clear(job, seg + 1, d);
    }
    TOC(6);
    // new segment
    had_base += nhad;
    nhad = 0;
    ++seg;
    open = false;
    if (is_meas) {
      if (job.dry) {
        // outcome-independent part of the filter: the dimension
        if (pend_r != 0) {
          uint64_t vj0[SF_WMAX];
          for (int w = 0; w < SF_WMAX; ++w) vj0[w] = L.V[pend_j0][w];
          __syncthreads();
          uint64_t mine[SF_WMAX];
          if (lane < d) for (int w = 0; w < SF_WMAX; ++w) mine[w] = L.V[lane][w] ^ (((pend_r >> lane) & 1u) ? vj0[w] : 0ull);
          __syncthreads();
          if (lane < d && lane != pend_j0) {
            int dst = lane < pend_j0 ? lane : lane - 1;
            for (int w = 0; w < SF_WMAX; ++w) L.V[dst][w] = mine[w];
          }
          d -= 1;
          __syncthreads();
        }
        pend = 0;
      } else {
        // the range ends at a measurement (the host splits ranges there)
        break;
      }
    }
    if (!job.dry) {
      for (int pt = lane; pt < SF_PMAX; pt += TL) L.acc[pt] = 0;
      build_points(L, d);
    }
    __syncthreads();
  }
  if (open && !job.dry && !err) {
    SegProg* sp = job.prog + seg;
    if (lane == 0) emit_header(sp, SEG_NONE, 0, d, d, nhad, had_base);
    if (rec) zero_z4(&sp->E);
    else fit_z4(L, L.acc, d, &sp->E, &err);
    zero_z4(&sp->B0);
    zero_z4(&sp->B1);
    ++seg;
  }
  __syncthreads();
  // write back
  for (int i = lane; i < n * SF_WMAX; i += TL) {
    st->rx[i] = L.rx[i];
    st->rz[i] = L.rz[i];
    st->cx[i] = L.cx[i];
    st->cz[i] = L.cz[i];
  }
  if (lane < SF_WMAX) st->s0[lane] = L.s0[lane];
  if (lane < d) for (int w = 0; w < SF_WMAX; ++w) st->V[lane][w] = L.V[lane][w];
  if (lane == 0) {
    st->d = d;
    st->nmeas = nmeas;
    st->pend = job.dry ? 0 : pend;
    st->pend_r = pend_r; st->pend_c0 = pend_c0; st->pend_j0 = pend_j0; st->pend_meas = pend_meas;
    st->dmax = dmax;
    if (err && !st->error) st->error = err;
    L.tc[7] += TCLOCK();
    for (int k = 0; k < 12; ++k) st->cycles[k] += L.tc[k];
  }
}

static __device__ void readout_body(Lds& L, int16_t* rank, const TrackState* st, const uint8_t* outcomes, ReadoutInfo* ri) {
  const int lane = lane_id();
  const int n = st->n;
  int d = st->d;
  for (int i = lane; i < SF_NMAX * SF_WMAX; i += TL) {
    L.rx[i] = i < n * SF_WMAX ? st->rx[i] : 0ull;
    L.rz[i] = i < n * SF_WMAX ? st->rz[i] : 0ull;
  }
  if (lane < SF_WMAX) L.s0[lane] = st->s0[lane];
  if (lane < d) for (int w = 0; w < SF_WMAX; ++w) L.V[lane][w] = st->V[lane][w];
  __syncthreads();
  if (st->pend) apply_pending(L, st, outcomes, &d);
  build_cols(L, n);
  rebuild_index(L, n);
  repair(L, n, d, false, 1);
  rebuild_index(L, n);
  for (int i = lane; i < n; i += TL) {
    int r = 0, li = L.lead[i];
    for (int j = 0; j < n; ++j) r += L.lead[j] < li;
    rank[i] = (int16_t)r;
  }
  __syncthreads();
  for (int i = lane; i < n; i += TL) {
    int r = rank[i];
    for (int w = 0; w < W; ++w) {
      ri->tab[(size_t)r * 2 * W + w] = L.rx[i * SF_WMAX + w];
      ri->tab[(size_t)r * 2 * W + W + w] = L.rz[i * SF_WMAX + w];
    }
  }
  // hull in canonical row order
  if (lane <= d) {
    const uint64_t* vec = lane < d ? L.V[lane] : L.s0;
    uint64_t out[SF_WMAX] = {0, 0, 0, 0};
    for (int i = 0; i < n; ++i)
      if (getb(vec, i)) flipb(out, rank[i]);
    for (int w = 0; w < SF_WMAX; ++w) {
      if (lane < d) ri->V[lane][w] = out[w];
      else ri->s0[w] = out[w];
      L.hbN[lane][w] = out[w];
    }
  }
  __syncthreads();
  // descending echelon pivots of span(V)
  int nr = 0;
  span_reduce(L.hbN, nullptr, d, (int*)L.ech, &nr);
  __syncthreads();
  if (lane == 0) {
    int hb[SF_DMAX];
    for (int a = 0; a < nr && a < SF_DMAX; ++a) hb[a] = (int)L.ech[a];
    for (int a = 0; a < nr; ++a)  // descending
      for (int b = a + 1; b < nr; ++b)
        if (hb[b] > hb[a]) { int t = hb[a]; hb[a] = hb[b]; hb[b] = t; }
    for (int a = 0; a < nr; ++a) ri->piv[a] = hb[a];
    ri->n = n; ri->W = W; ri->d = d; ri->pad = nr == d ? 0 : 1;
  }
}
};

// One kernel per word count W (= ceil(n / 64)), so that each gets its own
// register allocation.
// One frame: the range given by value.
template <int W>
__device__ __forceinline__ void track_w(const TrackJob& job) {
  if constexpr (W <= 2) {
    __shared__ typename Trk<W>::LL L;
    Trk<W>::track_body(L, job);
  } else {
    __shared__ Lds L;
    TrkL<W>::track_body(L, job);
  }
}

template <int W>
__global__ void __launch_bounds__(TL) sf_track_one(TrackJob one) {
  track_w<W>(one);
}

// Many frames of the same W: workgroup b runs jobs[b].
template <int W>
__global__ void __launch_bounds__(TL) sf_track_many(const TrackJob* __restrict__ jobs) {
  const TrackJob job = jobs[blockIdx.x];
  track_w<W>(job);
}

// Split form: the phase evaluation of the Clifford gates of a range, one
// wavefront per chunk of gates (blockIdx.x = chunk, blockIdx.y = frame).
template <int W>
__device__ __forceinline__ void phase_w(const TrackJob& job, int c) {
  if constexpr (W <= 2) {
    typedef typename Trk<W>::LL LT;
    __shared__ __align__(16) unsigned char raw[phase_lds_bytes<LT>()];
    LT& L = *reinterpret_cast<LT*>(raw);
    Trk<W>::phase_body(L, job, c);
  } else {
    __shared__ Lds L;
    TrkL<W>::phase_body(L, job, c);
  }
}

template <int W>
__global__ void __launch_bounds__(TL) sf_phase_one(TrackJob one) {
  phase_w<W>(one, (int)blockIdx.x);
}

template <int W>
__global__ void __launch_bounds__(TL) sf_phase_many(const TrackJob* __restrict__ jobs) {
  const TrackJob job = jobs[blockIdx.y];
  phase_w<W>(job, (int)blockIdx.x);
}

// ... and the fit of each segment's summed phase (blockIdx.x = segment).
struct NoLds {};
__device__ void fit_body(const TrackJob& job, int s) {
  __shared__ uint8_t f[SF_PMAX];
  if (s >= job.nseg || job.dry || !job.rec) return;
  SegProg* sp = job.prog + s;
  const int d = sp->d;
  int err = 0;
  if (d < 0 || d >= SF_DMAX || npoints(d) > job.pe) {
    if (lane_id() == 0) job.st->error = TRK_E_INTERNAL;
    return;
  }
  const int P = npoints(d);
  const uint32_t* acc = job.segacc + (size_t)s * job.pe;
  for (int p = lane_id(); p < P; p += TL) f[p] = (uint8_t)(acc[p] & 3u);
  __syncthreads();
  NoLds none;
  fit_z4(none, f, d, &sp->E, &err);
  err = wave_max(err);
  if (err && lane_id() == 0) job.st->error = err;
}

extern "C" __global__ void __launch_bounds__(TL) sf_fit_one(TrackJob one) { fit_body(one, (int)blockIdx.x); }

extern "C" __global__ void __launch_bounds__(TL) sf_fit_many(const TrackJob* __restrict__ jobs) {
  const TrackJob job = jobs[blockIdx.y];
  fit_body(job, (int)blockIdx.x);
}

// Readout: canonical (fully reduced, pivot-sorted) tableau, the hull in that
// row order, and the descending echelon pivots of the hull.
extern "C" __global__ void __launch_bounds__(TL)
sf_readout_track(const TrackState* st, const uint8_t* outcomes, ReadoutInfo* ri) {
  __shared__ Lds L;
  __shared__ int16_t rank[SF_NMAX];
  switch (st->W) {
    case 1: TrkL<1>::readout_body(L, rank, st, outcomes, ri); break;
    case 2: TrkL<2>::readout_body(L, rank, st, outcomes, ri); break;
    case 3: TrkL<3>::readout_body(L, rank, st, outcomes, ri); break;
    default: TrkL<4>::readout_body(L, rank, st, outcomes, ri); break;
  }
}
