// Element kernels: stream the dense amplitude array of a frame.
//
// Slot Y of the array holds the element (sigma(Y), amp[Y]) of the frame; the
// phase vectors themselves are implicit in the hull (sf_dev.h).  A segment
// kernel applies, per element, the global-phase factors of a run of Clifford
// gates (ROTATE with global-phase maintenance, section 3) and then the
// segment's terminal step: a deterministic phase, or COFACTOR with the
// non-Clifford phase on the |1> cofactor.  Cofactor children of partner
// elements (phase vectors differing by the rows that anticommute with Z_q)
// land on the same slot pair and are merged in place by a butterfly, so no
// sort is needed.  Measurement (section 4) reduces p(1) with a fixed-shape
// tree, draws a counter-based uniform and filters the consistent elements.
#include <hip/hip_runtime.h>

#include "sf_dev.h"

#define EB 256

__device__ __forceinline__ int evalZ4(const Z4Q* __restrict__ t, uint32_t Y) {
  int e = (int)t->c + __popc(t->L1 & Y) + 2 * __popc(t->L2 & Y);
  uint32_t m = Y & t->qnz;
  while (m) {
    int j = __builtin_ctz(m);
    m &= m - 1;
    e += 2 * (__popc(t->Q[j] & Y) & 1);
  }
  return e & 3;
}

__device__ __forceinline__ int evalGF2(const GF2Q* __restrict__ t, uint32_t Y) {
  int e = (int)t->c ^ (__popc(t->L & Y) & 1);
  uint32_t m = Y & t->qnz;
  while (m) {
    int j = __builtin_ctz(m);
    m &= m - 1;
    e ^= __popc(t->Q[j] & Y) & 1;
  }
  return e;
}

// a * exp(i pi m / 4)
__device__ __forceinline__ double2 rot8(double2 a, int m) {
  m &= 7;
  double r, i;
  switch (m >> 1) {
    case 0: r = a.x; i = a.y; break;
    case 1: r = -a.y; i = a.x; break;
    case 2: r = -a.x; i = -a.y; break;
    default: r = a.y; i = -a.x; break;
  }
  if (m & 1) {
    const double s = 0.70710678118654752440;
    double nr = __dmul_rn(__dsub_rn(r, i), s);
    double ni = __dmul_rn(__dadd_rn(r, i), s);
    r = nr; i = ni;
  }
  return make_double2(r, i);
}

__device__ __forceinline__ double2 cmul(double2 a, double re, double im) {
  return make_double2(__dsub_rn(__dmul_rn(a.x, re), __dmul_rn(a.y, im)),
                      __dadd_rn(__dmul_rn(a.x, im), __dmul_rn(a.y, re)));
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(__dadd_rn(a.x, b.x), __dadd_rn(a.y, b.y));
}

__device__ __forceinline__ double norm2(double2 a) {
  return __dadd_rn(__dmul_rn(a.x, a.x), __dmul_rn(a.y, a.y));
}

__device__ __forceinline__ double2 prune(double2 a) {
  return norm2(a) <= 1e-24 ? make_double2(0.0, 0.0) : a;
}

// accumulated global-phase exponent (units of pi/4) of the segment's Cliffords
__device__ __forceinline__ int seg_phase(const SegProg* __restrict__ sp, const GF2Q* __restrict__ had, uint32_t Y) {
  int m = 2 * evalZ4(&sp->E, Y) + sp->nhad;
  const int nh = sp->nhad;
  for (int h = 0; h < nh; ++h) m -= 2 * evalGF2(&had[h], Y);
  return m & 7;
}

// cofactor child x: a * 2^{-1/2} i^{B_x(Y)}
__device__ __forceinline__ double2 child(double2 a, const Z4Q* __restrict__ B, uint32_t Y) {
  double2 r = rot8(a, 2 * evalZ4(B, Y));
  const double s = 0.70710678118654752440;
  return make_double2(__dmul_rn(r.x, s), __dmul_rn(r.y, s));
}

// both control functionals of a direct controlled step read 1
__device__ __forceinline__ bool cond2(const SegProg* __restrict__ sp, uint32_t Y) {
  return ((sp->det_c ^ (uint32_t)__popc(sp->det_r & Y)) & (sp->det2_c ^ (uint32_t)__popc(sp->det2_r & Y)) & 1u) != 0;
}

__device__ __forceinline__ uint32_t insert_zero(uint64_t r, int j) {
  uint64_t lo = r & ((1ull << j) - 1ull);
  return (uint32_t)(lo | ((r >> j) << (j + 1)));
}

// A measurement of a qubit outside the Z block (section 4: cofactor on it,
// then keep one branch) whose cofactor adds a hull coordinate: the segment
// pass that would store both children is not run.  The measurement kernels
// compute a child from its parent element when they need it (grow_children:
// the operations of the SEG_GROW pass), which saves the write and re-read of
// the 2^(d+1) child slots.
__device__ __forceinline__ bool grow_meas(const SegProg* __restrict__ sp) {
  return sp->is_meas && sp->kind == SEG_GROW;
}

// ---------------------------------------------------------------------------
// Segment: Clifford phases, then the terminal step of the segment
// ---------------------------------------------------------------------------
__device__ __forceinline__ void seg_body(const SegProg* __restrict__ sp, const GF2Q* __restrict__ had_all,
                                         double2* __restrict__ amp, uint64_t tid, uint64_t stride) {
  if (grow_meas(sp)) return;  // folded into the measurement kernels
  const int kind = sp->kind;
  const int d = sp->d;
  const GF2Q* had = had_all + sp->had_off;
  const uint64_t N = 1ull << d;
  const double pre = sp->ph_re, pim = sp->ph_im;
  if (kind == SEG_PAIR) {
    const int j0 = sp->j0;
    const uint32_t delta = sp->delta;
    for (uint64_t r = tid; r < (N >> 1); r += stride) {
      uint32_t Y = insert_zero(r, j0);
      uint32_t Yd = Y ^ delta;
      double2 a = amp[Y], b = amp[Yd];
      a = rot8(a, seg_phase(sp, had, Y));
      b = rot8(b, seg_phase(sp, had, Yd));
      double2 c0 = cadd(child(a, &sp->B0, Y), child(b, &sp->B0, Yd));
      double2 c1 = cadd(child(a, &sp->B1, Y), child(b, &sp->B1, Yd));
      c1 = cmul(c1, pre, pim);
      amp[Y] = prune(c0);
      amp[Yd] = prune(c1);
    }
  } else if (kind == SEG_GROW) {
    for (uint64_t Y = tid; Y < N; Y += stride) {
      double2 a = amp[Y];
      a = rot8(a, seg_phase(sp, had, (uint32_t)Y));
      double2 c0 = child(a, &sp->B0, (uint32_t)Y);
      double2 c1 = cmul(child(a, &sp->B1, (uint32_t)Y), pre, pim);
      amp[Y] = prune(c0);
      amp[Y + N] = prune(c1);
    }
  } else if (kind == SEG_CX2P) {
    // elements with both controls 1 move to Y ^ delta with the factor
    // i^{B0(Y)}; a pair (Y, Y ^ delta) has equal control values, so the move
    // is a swap (delta = 0: a phase in place)
    const int j0 = sp->j0;
    const uint32_t delta = sp->delta;
    if (delta == 0) {
      for (uint64_t Y = tid; Y < N; Y += stride) {
        double2 a = amp[Y];
        if (a.x == 0.0 && a.y == 0.0) continue;
        a = rot8(a, seg_phase(sp, had, (uint32_t)Y));
        if (cond2(sp, (uint32_t)Y)) a = rot8(a, 2 * evalZ4(&sp->B0, (uint32_t)Y));
        amp[Y] = a;
      }
    } else {
      for (uint64_t r = tid; r < (N >> 1); r += stride) {
        const uint32_t Y = insert_zero(r, j0);
        const uint32_t Yd = Y ^ delta;
        double2 a = rot8(amp[Y], seg_phase(sp, had, Y));
        double2 b = rot8(amp[Yd], seg_phase(sp, had, Yd));
        if (cond2(sp, Y)) {
          amp[Y] = rot8(b, 2 * evalZ4(&sp->B0, Yd));
          amp[Yd] = rot8(a, 2 * evalZ4(&sp->B0, Y));
        } else {
          amp[Y] = a;
          amp[Yd] = b;
        }
      }
    }
  } else if (kind == SEG_CX2G) {
    // elements with both controls 1 move to the new half Y + 2^d
    for (uint64_t Y = tid; Y < N; Y += stride) {
      double2 a = rot8(amp[Y], seg_phase(sp, had, (uint32_t)Y));
      const double2 z = make_double2(0.0, 0.0);
      if (cond2(sp, (uint32_t)Y)) {
        amp[Y] = z;
        amp[Y + N] = rot8(a, 2 * evalZ4(&sp->B0, (uint32_t)Y));
      } else {
        amp[Y] = a;
        amp[Y + N] = z;
      }
    }
  } else {
    const uint32_t dc = sp->det_c, dr = sp->det_r;
    const bool det = kind == SEG_DET, det2 = kind == SEG_DET2;
    for (uint64_t Y = tid; Y < N; Y += stride) {
      double2 a = amp[Y];
      if (a.x == 0.0 && a.y == 0.0) continue;
      a = rot8(a, seg_phase(sp, had, (uint32_t)Y));
      if (det && ((dc ^ (uint32_t)__popc(dr & (uint32_t)Y)) & 1u)) a = cmul(a, pre, pim);
      if (det2 && cond2(sp, (uint32_t)Y)) a = cmul(a, pre, pim);
      amp[Y] = a;
    }
  }
}

// The two children the SEG_GROW pass would store for parent element a at
// slot Y < 2^d: child 0 at slot Y, child 1 at slot Y + 2^d.
__device__ __forceinline__ void grow_children(const SegProg* __restrict__ sp, const GF2Q* __restrict__ had_all,
                                              double2 a, uint32_t Y, double2* c0, double2* c1) {
  a = rot8(a, seg_phase(sp, had_all + sp->had_off, Y));
  *c0 = prune(child(a, &sp->B0, Y));
  *c1 = prune(cmul(child(a, &sp->B1, Y), sp->ph_re, sp->ph_im));
}

// ... and the one at child slot Yc < 2^(d+1) (parent element a = amp[Yc mod 2^d])
__device__ __forceinline__ double2 grow_child_of(const SegProg* __restrict__ sp, const GF2Q* __restrict__ had_all,
                                                 double2 a, uint64_t Yc) {
  const uint64_t N = 1ull << sp->d;
  const uint32_t Y = (uint32_t)(Yc & (N - 1));
  a = rot8(a, seg_phase(sp, had_all + sp->had_off, Y));
  if (Yc < N) return prune(child(a, &sp->B0, Y));
  return prune(cmul(child(a, &sp->B1, Y), sp->ph_re, sp->ph_im));
}

// Reduction shape of a measurement over 2^d slots: red_grid(d) blocks of EB
// threads, about SF_RED_EPT slots per thread (at most SF_RED_GMAX blocks).
// A function of d alone, so every path (one frame, batched, graph) adds the
// same terms in the same order.
#define SF_RED_EPT 8
#define SF_RED_GMAX 1024
__host__ __device__ __forceinline__ int red_grid(int d) {
  const uint64_t per = (uint64_t)EB * SF_RED_EPT;
  const uint64_t g = ((1ull << d) + per - 1) / per;
  return g > SF_RED_GMAX ? SF_RED_GMAX : (int)g;
}

__device__ __forceinline__ void meas_acc(double2 a, uint64_t Y, uint32_t c0, uint32_t r, double& p0, double& p1) {
  const double v = norm2(a);
  if ((c0 ^ (uint32_t)__popc(r & (uint32_t)Y)) & 1u) p1 = __dadd_rn(p1, v);
  else p0 = __dadd_rn(p0, v);
}

// A growing measurement's per-thread sums: thread t of block b takes the
// parents Y = b*EB + t + m*G*EB < 2^d in turn and adds child 0 (slot Y), then
// child 1 (slot Y + 2^d), each parent read once (four loads in flight).
__device__ __forceinline__ void grow_meas_acc(const SegProg* __restrict__ sp, const GF2Q* __restrict__ had_all,
                                              const double2* __restrict__ amp, int block, int G, double& p0,
                                              double& p1) {
  const uint64_t N = 1ull << sp->d;
  const uint32_t c0 = sp->m_c0, r = sp->m_r;
  const uint64_t stride = (uint64_t)G * EB;
  uint64_t Y = (uint64_t)block * EB + threadIdx.x;
  for (; Y + 3 * stride < N; Y += 4 * stride) {
    double2 a[4];
    for (int m = 0; m < 4; ++m) a[m] = amp[Y + m * stride];
    for (int m = 0; m < 4; ++m) {
      const uint64_t Ym = Y + m * stride;
      double2 ch0, ch1;
      grow_children(sp, had_all, a[m], (uint32_t)Ym, &ch0, &ch1);
      meas_acc(ch0, Ym, c0, r, p0, p1);
      meas_acc(ch1, Ym + N, c0, r, p0, p1);
    }
  }
  for (; Y < N; Y += stride) {
    double2 ch0, ch1;
    grow_children(sp, had_all, amp[Y], (uint32_t)Y, &ch0, &ch1);
    meas_acc(ch0, Y, c0, r, p0, p1);
    meas_acc(ch1, Y + N, c0, r, p0, p1);
  }
}

// Measurement: block partial sums of |a|^2 split by the qubit value; block b
// of G = red_grid(d) covers slots b*EB + t, stepping by G*EB, in that order,
// then a pairwise tree over the block's threads (s[t] += s[t + h] for
// h = EB/2 .. 1; the levels within one wavefront by lane shuffles, which add
// the same pairs).  Blocks b >= G write nothing.
__device__ __forceinline__ void meas_reduce_body(const SegProg* __restrict__ sp, const GF2Q* __restrict__ had_all,
                                                 const double2* __restrict__ amp, double2* __restrict__ partials,
                                                 int block) {
  __shared__ double s0[EB], s1[EB];
  const int d = sp->d_out;
  const int G = red_grid(d);
  if (block >= G) return;
  const uint64_t N = 1ull << d;
  const uint32_t c0 = sp->m_c0, r = sp->m_r;
  const uint64_t stride = (uint64_t)G * EB;
  double p0 = 0.0, p1 = 0.0;
  uint64_t Y = (uint64_t)block * EB + threadIdx.x;
  if (grow_meas(sp)) {
    grow_meas_acc(sp, had_all, amp, block, G, p0, p1);
    Y = N;
  }
  // four loads in flight, added in slot order
  for (; Y + 3 * stride < N; Y += 4 * stride) {
    const double2 a0 = amp[Y], a1 = amp[Y + stride], a2 = amp[Y + 2 * stride], a3 = amp[Y + 3 * stride];
    meas_acc(a0, Y, c0, r, p0, p1);
    meas_acc(a1, Y + stride, c0, r, p0, p1);
    meas_acc(a2, Y + 2 * stride, c0, r, p0, p1);
    meas_acc(a3, Y + 3 * stride, c0, r, p0, p1);
  }
  for (; Y < N; Y += stride) meas_acc(amp[Y], Y, c0, r, p0, p1);
  s0[threadIdx.x] = p0;
  s1[threadIdx.x] = p1;
  __syncthreads();
  for (int h = EB / 2; h >= 64; h >>= 1) {
    if (threadIdx.x < h) {
      s0[threadIdx.x] = __dadd_rn(s0[threadIdx.x], s0[threadIdx.x + h]);
      s1[threadIdx.x] = __dadd_rn(s1[threadIdx.x], s1[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 64) {
    double v0 = s0[threadIdx.x], v1 = s1[threadIdx.x];
    for (int h = 32; h > 0; h >>= 1) {
      const double u0 = __shfl_down(v0, h, 64), u1 = __shfl_down(v1, h, 64);
      v0 = __dadd_rn(v0, u0);
      v1 = __dadd_rn(v1, u1);
    }
    if (threadIdx.x == 0) partials[block] = make_double2(v0, v1);
  }
}

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t state, uint64_t index) {
  // output `index` of the SplitMix64 generator started at `state`
  uint64_t z = state + (index + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The coin inside each filter block: the sum of the partials in the one-block
// shape of the final step (slot t of EB adds partials t, t + EB, ... in
// order, then the pairwise tree; the block's threads share the slots, and
// within a tree level the additions are independent), the seeded coin and
// the scale.  Every block computes the same values; the writer block stores
// them.  One launch less per measurement than a separate coin kernel.
__device__ __forceinline__ void meas_coin_local(const SegProg* __restrict__ sp, const double2* __restrict__ partials,
                                                uint64_t seed, bool writer, uint8_t* __restrict__ outcomes,
                                                double* __restrict__ pvals, double* __restrict__ scale,
                                                int* __restrict__ flags, uint32_t* o_out, double* sc_out) {
  __shared__ double v0[EB], v1[EB];
  __shared__ uint32_t s_o;
  __shared__ double s_sc;
  const int nt = blockDim.x;
  const int G = red_grid(sp->d_out);
  for (int t = threadIdx.x; t < EB; t += nt) {
    double p0 = 0.0, p1 = 0.0;
    for (int i = t; i < G; i += EB) {
      p0 = __dadd_rn(p0, partials[i].x);
      p1 = __dadd_rn(p1, partials[i].y);
    }
    v0[t] = p0;
    v1[t] = p1;
  }
  __syncthreads();
  for (int h = EB / 2; h > 0; h >>= 1) {
    for (int t = threadIdx.x; t < h; t += nt) {
      v0[t] = __dadd_rn(v0[t], v0[t + h]);
      v1[t] = __dadd_rn(v1[t], v1[t + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int mi = sp->meas_index;
    double P0 = v0[0], P1 = v1[0];
    double u = (double)(splitmix64_at(seed, (uint64_t)mi) >> 11) * (1.0 / 9007199254740992.0);
    int o = u < P1 ? 1 : 0;
    double po = o ? P1 : P0;
    const double sc = po > 0.0 ? 1.0 / sqrt(po) : 0.0;
    if (writer) {
      outcomes[mi] = (uint8_t)o;
      pvals[mi] = P1;
      scale[0] = sc;
      if (fabs(u - P1) < 1e-12 || po <= 0.0) atomicOr(flags, 1);
    }
    s_o = (uint32_t)o;
    s_sc = sc;
  }
  __syncthreads();
  *o_out = s_o;
  *sc_out = s_sc;
}

// Keep the elements consistent with the outcome and renormalise (new buffer).
__device__ __forceinline__ void meas_filter_body(const SegProg* __restrict__ sp, const GF2Q* __restrict__ had_all,
                                                 const double2* __restrict__ src, double2* __restrict__ dst,
                                                 uint32_t o, double s, uint64_t tid, uint64_t stride) {
  const uint32_t c0 = sp->m_c0, r = sp->m_r;
  const int j0 = sp->m_j0;
  const int dout = sp->d_out;
  if (grow_meas(sp)) {
    // kept slot Yp holds child slot Y (below): computed from its parent,
    // four parent loads in flight
    const uint64_t Np = 1ull << sp->d;
    const uint64_t N = r ? (1ull << (dout - 1)) : (1ull << dout);
    for (uint64_t Y0 = tid; Y0 < N; Y0 += 4 * stride) {
      uint32_t Ys[4];
      double2 a[4];
      for (int m = 0; m < 4; ++m) {
        const uint64_t Yp = Y0 + m * stride;
        uint32_t Y = (uint32_t)Yp;
        if (r) {
          const uint32_t rest = insert_zero(Yp, j0);
          Y = rest | (((o ^ c0 ^ (uint32_t)__popc(r & rest)) & 1u) << j0);
        }
        Ys[m] = Y;
        a[m] = Yp < N ? src[Y & (Np - 1)] : make_double2(0.0, 0.0);
      }
      for (int m = 0; m < 4; ++m) {
        const uint64_t Yp = Y0 + m * stride;
        if (Yp >= N) break;
        const double2 v = grow_child_of(sp, had_all, a[m], Ys[m]);
        dst[Yp] = make_double2(__dmul_rn(v.x, s), __dmul_rn(v.y, s));
      }
    }
    return;
  }
  if (r == 0) {
    const uint64_t N = 1ull << dout;
    for (uint64_t Y = tid; Y < N; Y += stride) {
      double2 a = src[Y];
      dst[Y] = make_double2(__dmul_rn(a.x, s), __dmul_rn(a.y, s));
    }
  } else {
    const uint64_t N = 1ull << (dout - 1);
    for (uint64_t Yp = tid; Yp < N; Yp += stride) {
      uint32_t rest = insert_zero(Yp, j0);
      uint32_t bit = (o ^ c0 ^ (uint32_t)__popc(r & rest)) & 1u;
      double2 a = src[rest | (bit << j0)];
      dst[Yp] = make_double2(__dmul_rn(a.x, s), __dmul_rn(a.y, s));
    }
  }
}

// Frames of at most EB slots (hull dimension <= 8 for the whole circuit, so
// one reduction block, G = 1): reduction, coin and filter of a measurement in
// one block.  The sums equal those of the three-kernel form: the single
// block's tree gives the only non-zero partial, and the final pass adds only
// +0.0 to it (exact for a non-negative sum).
__device__ __forceinline__ void meas_small_body(const SegProg* __restrict__ sp, const GF2Q* __restrict__ had_all,
                                                const double2* __restrict__ src, double2* __restrict__ dst, uint64_t seed,
                                                uint8_t* __restrict__ outcomes, double* __restrict__ pvals,
                                                double* __restrict__ scale, int* __restrict__ flags) {
  __shared__ double s0[EB], s1[EB];
  __shared__ double s_scale;
  __shared__ uint32_t s_out;
  const uint64_t N = 1ull << sp->d_out;
  const uint32_t c0 = sp->m_c0, r = sp->m_r;
  const bool gm = grow_meas(sp);
  double p0 = 0.0, p1 = 0.0;
  if (gm) grow_meas_acc(sp, had_all, src, 0, 1, p0, p1);  // the one-block shape of the reduction
  else
    for (uint64_t Y = threadIdx.x; Y < N; Y += EB) meas_acc(src[Y], Y, c0, r, p0, p1);
  s0[threadIdx.x] = p0;
  s1[threadIdx.x] = p1;
  __syncthreads();
  for (int h = EB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      s0[threadIdx.x] = __dadd_rn(s0[threadIdx.x], s0[threadIdx.x + h]);
      s1[threadIdx.x] = __dadd_rn(s1[threadIdx.x], s1[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int mi = sp->meas_index;
    double P0 = __dadd_rn(0.0, s0[0]), P1 = __dadd_rn(0.0, s1[0]);
    double u = (double)(splitmix64_at(seed, (uint64_t)mi) >> 11) * (1.0 / 9007199254740992.0);
    int o = u < P1 ? 1 : 0;
    outcomes[mi] = (uint8_t)o;
    pvals[mi] = P1;
    double po = o ? P1 : P0;
    const double sc = po > 0.0 ? 1.0 / sqrt(po) : 0.0;
    scale[0] = sc;
    if (fabs(u - P1) < 1e-12 || po <= 0.0) atomicOr(flags, 1);
    s_out = (uint32_t)o;
    s_scale = sc;
  }
  __syncthreads();
  const uint32_t o = s_out;
  const double sc = s_scale;
  const int j0 = sp->m_j0;
  const int dout = sp->d_out;
  const uint64_t Np = gm ? (1ull << sp->d) : N;
  if (r == 0) {
    for (uint64_t Y = threadIdx.x; Y < N; Y += EB) {
      double2 a = gm ? grow_child_of(sp, had_all, src[Y & (Np - 1)], Y) : src[Y];
      dst[Y] = make_double2(__dmul_rn(a.x, sc), __dmul_rn(a.y, sc));
    }
  } else {
    const uint64_t Nh = 1ull << (dout - 1);
    for (uint64_t Yp = threadIdx.x; Yp < Nh; Yp += EB) {
      uint32_t rest = insert_zero(Yp, j0);
      uint32_t bit = (o ^ c0 ^ (uint32_t)__popc(r & rest)) & 1u;
      const uint32_t Y = rest | (bit << j0);
      double2 a = gm ? grow_child_of(sp, had_all, src[Y & (Np - 1)], Y) : src[Y];
      dst[Yp] = make_double2(__dmul_rn(a.x, sc), __dmul_rn(a.y, sc));
    }
  }
}

#define TID ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x)
#define STRIDE ((uint64_t)gridDim.x * blockDim.x)

extern "C" __global__ void __launch_bounds__(EB)
sf_seg_kernel(const SegProg* __restrict__ sp, const GF2Q* __restrict__ had_all, double2* __restrict__ amp) {
  seg_body(sp, had_all, amp, TID, STRIDE);
}

extern "C" __global__ void __launch_bounds__(EB)
sf_meas_reduce(const SegProg* __restrict__ sp, const GF2Q* __restrict__ had_all, const double2* __restrict__ amp,
               double2* __restrict__ partials) {
  meas_reduce_body(sp, had_all, amp, partials, blockIdx.x);
}

extern "C" __global__ void __launch_bounds__(EB)
sf_meas_filter(const SegProg* __restrict__ sp, const GF2Q* __restrict__ had_all,
               const double2* __restrict__ partials, uint64_t seed,
               uint8_t* __restrict__ outcomes, double* __restrict__ pvals, double* __restrict__ scale,
               int* __restrict__ flags, const double2* __restrict__ src, double2* __restrict__ dst) {
  uint32_t o;
  double sc;
  meas_coin_local(sp, partials, seed, blockIdx.x == 0, outcomes, pvals, scale, flags, &o, &sc);
  meas_filter_body(sp, had_all, src, dst, o, sc, TID, STRIDE);
}

// ---------------------------------------------------------------------------
// Batched forms, flattened: the grid is the concatenation of every frame's
// blocks.  B[j] is the first block of frame j's descriptor (B[0] = 0, B[na] =
// the grid); a frame without blocks in a launch is idle there.  A segment
// launch takes its row k (the program at prog + k), the measurement
// launches the frame's measurement program (prog + mk).  A block finds its frame by a
// binary search over B (uniform across the block) and strides over that
// frame's slots with the frame's own block count, so each frame launches
// only the blocks its hull needs.
// ---------------------------------------------------------------------------
struct BatchPos {
  int j;            // descriptor
  uint64_t tid;     // thread index within the frame's blocks
  uint64_t stride;  // threads of the frame's blocks
  uint32_t blk;     // block index within the frame's blocks
};

__device__ __forceinline__ BatchPos batch_pos(const uint32_t* __restrict__ B, int na) {
  const uint32_t b = blockIdx.x;
  int lo = 0, hi = na;  // B[lo] <= b < B[hi] (B[na] is the grid)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (B[mid] <= b) lo = mid;
    else hi = mid;
  }
  BatchPos p;
  p.j = lo;
  const uint32_t b0 = B[lo];
  const uint32_t nb = B[lo + 1] - b0;
  p.blk = b - b0;
  p.tid = (uint64_t)p.blk * blockDim.x + threadIdx.x;
  p.stride = (uint64_t)nb * blockDim.x;
  return p;
}

extern "C" __global__ void __launch_bounds__(EB)
sf_seg_batch(const ElemDesc* __restrict__ D, const uint32_t* __restrict__ B, int na, int k) {
  const BatchPos p = batch_pos(B, na);
  const ElemDesc& e = D[p.j];
  if (k >= e.nseg) return;
  seg_body(e.prog + k, e.had, e.amp, p.tid, p.stride);
}

// Reduction blocks of a frame: partial b of the shape red_grid(d) (the host
// launches red_grid of its bound on d; blocks beyond the actual shape exit).
extern "C" __global__ void __launch_bounds__(EB)
sf_meas_reduce_batch(const ElemDesc* __restrict__ D, const uint32_t* __restrict__ B, int na) {
  const BatchPos p = batch_pos(B, na);
  const ElemDesc& e = D[p.j];
  if (e.mk < 0) return;
  meas_reduce_body(e.prog + e.mk, e.had, e.amp, e.partials, (int)p.blk);
}

extern "C" __global__ void __launch_bounds__(EB)
sf_meas_filter_batch(const ElemDesc* __restrict__ D, const uint32_t* __restrict__ B, int na) {
  const BatchPos p = batch_pos(B, na);
  const ElemDesc& e = D[p.j];
  if (e.mk < 0) return;
  const SegProg* sp = e.prog + e.mk;
  uint32_t o;
  double sc;
  meas_coin_local(sp, e.partials, e.seedp ? *e.seedp : e.seed, p.blk == 0, e.outcomes, e.pvals,
                  e.scale, e.flags, &o, &sc);
  meas_filter_body(sp, e.had, e.amp, e.amp_other, o, sc, p.tid, p.stride);
}

// The same in two kernels for launches of many frames: the coin once per
// frame (one block each: the sums, outcome, p(1) and scale of
// meas_coin_local, stored), then the filter reading outcome and scale back.
// Same values as the fused kernel, without every filter block summing the
// partials again.
extern "C" __global__ void __launch_bounds__(EB) sf_meas_coin_batch(const ElemDesc* __restrict__ D) {
  const ElemDesc& e = D[blockIdx.x];
  if (e.mk < 0) return;
  uint32_t o;
  double sc;
  meas_coin_local(e.prog + e.mk, e.partials, e.seedp ? *e.seedp : e.seed, true, e.outcomes, e.pvals, e.scale,
                  e.flags, &o, &sc);
}

extern "C" __global__ void __launch_bounds__(EB)
sf_meas_apply_batch(const ElemDesc* __restrict__ D, const uint32_t* __restrict__ B, int na) {
  const BatchPos p = batch_pos(B, na);
  const ElemDesc& e = D[p.j];
  if (e.mk < 0) return;
  const SegProg* sp = e.prog + e.mk;
  const uint32_t o = e.outcomes[sp->meas_index];
  const double sc = e.scale[0];
  meas_filter_body(sp, e.had, e.amp, e.amp_other, o, sc, p.tid, p.stride);
}

// Frames of at most EB slots: every segment of a round, then its
// measurement, in one block per frame (segments in order, a barrier between
// them; each slot's arithmetic is that of the separate launches).
extern "C" __global__ void __launch_bounds__(EB)
sf_elem_small(const SegProg* __restrict__ prog, int nseg, const GF2Q* __restrict__ had_all,
              double2* __restrict__ amp, double2* __restrict__ amp_other, int meas, uint64_t seed,
              uint8_t* __restrict__ outcomes, double* __restrict__ pvals, double* __restrict__ scale,
              int* __restrict__ flags) {
  for (int k = 0; k < nseg; ++k) {
    seg_body(prog + k, had_all, amp, threadIdx.x, EB);
    __syncthreads();
  }
  if (meas) meas_small_body(prog + (nseg - 1), had_all, amp, amp_other, seed, outcomes, pvals, scale, flags);
}

// batched form: block j = frame j (descriptor j): its segments k < nseg in
// order, then its measurement if it has one
extern "C" __global__ void __launch_bounds__(EB)
sf_elem_small_batch(const ElemDesc* __restrict__ D, int kmax, int na, int meas) {
  const int j = blockIdx.x;
  for (int k = 0; k < kmax; ++k) {
    const ElemDesc& e = D[j];
    if (k < e.nseg) seg_body(e.prog + k, e.had, e.amp, threadIdx.x, EB);
    __syncthreads();
  }
  if (!meas) return;
  const ElemDesc& e = D[j];
  if (e.mk < 0) return;
  meas_small_body(e.prog + e.mk, e.had, e.amp, e.amp_other, e.seedp ? *e.seedp : e.seed, e.outcomes, e.pvals, e.scale,
                  e.flags);
}

// Number of non-zero amplitudes (frame size |F|).
extern "C" __global__ void __launch_bounds__(EB)
sf_count_kernel(const TrackState* __restrict__ st, const double2* __restrict__ amp, unsigned long long* out) {
  __shared__ unsigned long long sc[EB];
  // a measurement's filter is already applied to the array, not yet to the hull
  const int d = st->d - ((st->pend && st->pend_r) ? 1 : 0);
  const uint64_t N = 1ull << d;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  unsigned long long c = 0;
  for (uint64_t Y = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; Y < N; Y += stride) {
    double2 a = amp[Y];
    c += (a.x != 0.0 || a.y != 0.0) ? 1ull : 0ull;
  }
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int h = EB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) sc[threadIdx.x] += sc[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && sc[0]) atomicAdd(out, sc[0]);
}

// ---------------------------------------------------------------------------
// Readout in canonical order
// ---------------------------------------------------------------------------
// Scatter every slot to its rank key: the phase-vector bits at the echelon
// pivots of the hull, which orders slots exactly as ascending sigma.
extern "C" __global__ void __launch_bounds__(EB)
sf_readout_scatter(const ReadoutInfo* __restrict__ ri, const double2* __restrict__ amp,
                   uint64_t* __restrict__ tsig, double2* __restrict__ tamp, uint8_t* __restrict__ flag) {
  const int d = ri->d, W = ri->W;
  const uint64_t N = 1ull << d;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t Y = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; Y < N; Y += stride) {
    uint64_t s[SF_WMAX];
    for (int w = 0; w < SF_WMAX; ++w) s[w] = ri->s0[w];
    uint32_t y = (uint32_t)Y;
    while (y) {
      int j = __builtin_ctz(y);
      y &= y - 1;
      for (int w = 0; w < SF_WMAX; ++w) s[w] ^= ri->V[j][w];
    }
    uint64_t key = 0;
    for (int i = 0; i < d; ++i) {
      int pv = ri->piv[i];
      key = (key << 1) | ((s[pv >> 6] >> (pv & 63)) & 1ull);
    }
    double2 a = amp[Y];
    for (int w = 0; w < W; ++w) tsig[key * W + w] = s[w];
    tamp[key] = a;
    flag[key] = (a.x != 0.0 || a.y != 0.0) ? 1 : 0;
  }
}

#define CH_ITEMS 16
#define CH (EB * CH_ITEMS)

extern "C" __global__ void __launch_bounds__(EB)
sf_compact_count(const uint8_t* __restrict__ flag, uint64_t N, unsigned int* __restrict__ counts) {
  __shared__ unsigned int sc[EB];
  uint64_t base = (uint64_t)blockIdx.x * CH + (uint64_t)threadIdx.x * CH_ITEMS;
  unsigned int c = 0;
  for (int k = 0; k < CH_ITEMS; ++k) c += (base + k < N) ? flag[base + k] : 0u;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int h = EB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) sc[threadIdx.x] += sc[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = sc[0];
}

// single block: exclusive scan of the block counts, total at counts[nb]
extern "C" __global__ void __launch_bounds__(EB)
sf_compact_scan(unsigned int* __restrict__ counts, int nb, unsigned long long* __restrict__ total) {
  __shared__ unsigned long long part[EB];
  const int per = (nb + EB - 1) / EB;
  const int b0 = threadIdx.x * per;
  unsigned long long s = 0;
  for (int i = 0; i < per; ++i) if (b0 + i < nb) s += counts[b0 + i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int t = 0; t < EB; ++t) { unsigned long long v = part[t]; part[t] = run; run += v; }
    *total = run;
  }
  __syncthreads();
  unsigned long long run = part[threadIdx.x];
  for (int i = 0; i < per; ++i) {
    if (b0 + i < nb) { unsigned int v = counts[b0 + i]; counts[b0 + i] = (unsigned int)run; run += v; }
  }
}

extern "C" __global__ void __launch_bounds__(EB)
sf_compact_write(const uint8_t* __restrict__ flag, const uint64_t* __restrict__ tsig, const double2* __restrict__ tamp,
                 uint64_t N, int W, const unsigned int* __restrict__ offs, uint64_t* __restrict__ osig,
                 double2* __restrict__ oamp) {
  __shared__ unsigned int sc[EB];
  uint64_t base = (uint64_t)blockIdx.x * CH + (uint64_t)threadIdx.x * CH_ITEMS;
  unsigned int c = 0;
  for (int k = 0; k < CH_ITEMS; ++k) c += (base + k < N) ? flag[base + k] : 0u;
  sc[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int run = 0;
    for (int t = 0; t < EB; ++t) { unsigned int v = sc[t]; sc[t] = run; run += v; }
  }
  __syncthreads();
  uint64_t pos = (uint64_t)offs[blockIdx.x] + sc[threadIdx.x];
  for (int k = 0; k < CH_ITEMS; ++k) {
    uint64_t i = base + k;
    if (i < N && flag[i]) {
      for (int w = 0; w < W; ++w) osig[pos * W + w] = tsig[i * W + w];
      oamp[pos] = tamp[i];
      ++pos;
    }
  }
}

// Basis state |b>: stabilizer matrix in basis form (row q = Z_q, Figure 2a),
// phase vector sigma = b, one element of amplitude 1.
__device__ void init_body(TrackState* __restrict__ st, int n, uint64_t b0, uint64_t b1, uint64_t b2, uint64_t b3,
                          double2* __restrict__ amp, int* __restrict__ flags) {
  const int W = (n + 63) / 64;
  // (slots and qubits from n on are never read: every reader masks them)
  for (int i = threadIdx.x; i < n * SF_WMAX; i += blockDim.x) {
    int q = i / SF_WMAX, w = i % SF_WMAX;
    const uint64_t z = w == (q >> 6) ? (1ull << (q & 63)) : 0ull;
    st->rx[i] = 0ull;
    st->rz[i] = z;
    st->cx[i] = 0ull;
    st->cz[i] = z;  // the basis form is its own transpose
  }
  if (threadIdx.x == 0) {
    st->n = n; st->W = W; st->d = 0; st->nmeas = 0;
    st->pend = 0; st->pend_j0 = -1; st->pend_c0 = 0; st->pend_meas = -1; st->pend_r = 0;
    st->dmax = 0; st->error = 0; st->pad = 0;
    for (int k = 0; k < 16; ++k) st->cycles[k] = 0;
    uint64_t b[4] = {b0, b1, b2, b3};
    for (int w = 0; w < SF_WMAX; ++w) {
      uint64_t m = w < W ? ~0ull : 0ull;
      if (w == W - 1 && (n & 63)) m = (1ull << (n & 63)) - 1ull;
      st->s0[w] = b[w] & m;
    }
    amp[0] = make_double2(1.0, 0.0);
    *flags = 0;
  }
}

extern "C" __global__ void __launch_bounds__(EB)
sf_init_state(TrackState* __restrict__ st, int n, uint64_t b0, uint64_t b1, uint64_t b2, uint64_t b3,
              double2* __restrict__ amp, int* __restrict__ flags) {
  init_body(st, n, b0, b1, b2, b3, amp, flags);
}

// One block per frame (blockIdx.x selects the InitDesc).
extern "C" __global__ void __launch_bounds__(EB) sf_init_batch(const InitDesc* __restrict__ D) {
  const InitDesc& e = D[blockIdx.x];
  const uint64_t* b = e.params;
  init_body(e.st, e.n, b[0], b[1], b[2], b[3], e.amp, e.flags);
}

// Unit amplitudes over N slots (scratch input of the autotuner).
extern "C" __global__ void __launch_bounds__(EB) sf_fill_unit(double2* __restrict__ amp, uint64_t N) {
  for (uint64_t i = TID; i < N; i += STRIDE) amp[i] = make_double2(1.0, 0.0);
}

// Error words of many tableau tracks in one launch (out[i] = sts[i]->error).
extern "C" __global__ void __launch_bounds__(EB)
sf_gather_errors(const TrackState* const* __restrict__ sts, int n, int* __restrict__ out) {
  for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < n; i += (int)(gridDim.x * blockDim.x))
    out[i] = sts[i]->error;
}
