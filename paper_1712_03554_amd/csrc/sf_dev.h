// Device-side data layout of the stabilizer-frame engine (gfx950).
//
// A frame (Definition 1 of Garcia & Markov) is held as
//   * the stabilizer matrix: n slots of (x, z) bit rows, kept in the
//     row-echelon form of Figure 2b (X-block rows reduced on their x-leads,
//     Z-block rows reduced on their z-leads); slot i owns phase-vector bit i;
//   * the affine hull of the phase vectors: sigma(Y) = s0 ^ XOR_{j in Y} V[j],
//     Y in [0, 2^d);
//   * a dense array amp[Y] (complex128); slot Y holds the element
//     (sigma(Y), amp[Y]) and amp[Y] == 0 means "no element".
// Every phase-vector operation of the paper (sign flips, memoised row
// operations, cofactor children) is applied to s0 and V only; per element the
// engine updates amplitudes through per-segment phase programs.
#pragma once
#include <stdint.h>

#define SF_NMAX 256          // qubits
#define SF_WMAX 4            // 64-bit words per packed row
#define SF_DMAX 30           // hull dimension (2^30 amplitudes per buffer)
#define SF_PMAX (1 + SF_DMAX + SF_DMAX * (SF_DMAX - 1) / 2)

// device gate codes (after load-time rewriting)
// DG_NCPHASE and later codes end a segment: a non-Clifford phase (a split),
// a measurement, and the last step of a direct controlled phase (DG_CPH2:
// phase on the elements where q0 and q1 read 1) or direct Toffoli (DG_CX2: X
// on q2 for the elements where q0 and q1 read 1), both after cofactors on
// their two controls.
enum { DG_H = 0, DG_S, DG_SDG, DG_X, DG_Y, DG_Z, DG_CNOT, DG_CZ, DG_NCPHASE, DG_MEASURE, DG_CPH2, DG_CX2 };

struct DGate {            // 32 bytes
  int32_t op, q0, q1, q2;
  double c, s;            // exp(i theta) of a non-Clifford phase gate
};

// Z4-valued quadratic function of the hull coordinates:
//   e(Y) = c + popc(L1&Y) + 2 popc(L2&Y) + 2 sum_{j in Y & qnz} parity(Q[j] & Y)   (mod 4)
// Q[j] holds coefficients of Y_j Y_j' for j' > j only.
struct Z4Q {
  uint32_t c, L1, L2, qnz;
  uint32_t Q[32];
};
// GF(2)-valued quadratic function: t(Y) = c ^ parity(L&Y) ^ sum_{j in Y & qnz} parity(Q[j]&Y)
struct GF2Q {
  uint32_t c, L, qnz, pad;
  uint32_t Q[32];
};

enum { SEG_NONE = 0, SEG_DET = 1, SEG_GROW = 2, SEG_PAIR = 3,
       SEG_DET2 = 4,   // phase on the elements where two qubit functionals read 1
       SEG_CX2P = 5,   // those elements move to Y ^ delta (delta = 0: stay) with factor i^{B0(Y)}
       SEG_CX2G = 6 }; // those elements move to Y + 2^d with factor i^{B0(Y)}

// Program of one segment: a run of Clifford gates (folded phase E plus one
// GF(2) term per Hadamard whose support size is unchanged) followed by at most
// one terminal step (non-Clifford phase gate, measurement, or the last step of
// a direct controlled phase / Toffoli).
struct SegProg {
  int32_t kind;        // SEG_*
  int32_t is_meas;
  int32_t d;           // hull dimension on entry
  int32_t d_out;       // after the split
  int32_t nhad;        // GF(2) terms of this segment
  int32_t had_off;     // index of the first one in the had-term array
  int32_t j0;          // SEG_PAIR: coordinate whose pairs merge
  uint32_t delta;      // SEG_PAIR: partner offset
  uint32_t det_c, det_r;   // SEG_DET: qubit value x(Y) = det_c ^ parity(det_r & Y)
  uint32_t m_c0, m_r;      // measurement: qubit value after the split
  int32_t m_j0;            // highest set bit of m_r, or -1
  int32_t meas_index;
  int32_t nhad_total;      // odd part count (number of Hadamard half-steps)
  uint32_t det2_c, det2_r; // SEG_DET2 / SEG_CX2*: second qubit functional
  int32_t pad;
  double ph_re, ph_im;     // exp(i theta) on the |1> branch
  Z4Q E;                   // folded Clifford phase exponent (units of i)
  Z4Q B0, B1;              // split children: beta_x = 2^{-1/2} i^{B_x(Y)}
};

// Persistent per-frame tableau/hull state in device memory.
struct TrackState {
  int32_t n, W, d, nmeas;
  int32_t pend, pend_j0, pend_c0, pend_meas;
  uint32_t pend_r;
  int32_t dmax, error, pad;
  uint64_t rx[SF_NMAX * SF_WMAX];
  uint64_t rz[SF_NMAX * SF_WMAX];
  // column-major copy kept with the rows: cx / cz at qubit q hold the slots
  // whose row has an x / z bit there
  uint64_t cx[SF_NMAX * SF_WMAX];
  uint64_t cz[SF_NMAX * SF_WMAX];
  uint64_t s0[SF_WMAX];
  uint64_t V[SF_DMAX][SF_WMAX];
  uint64_t cycles[16];     // shader clocks spent per phase of the track (profiling)
};

// One circuit range for the tableau-track kernel.
//
// Split form (frames of up to 128 qubits): the track kernel only conjugates,
// repairs and records the state after every gate (rec: g1 - g0 + 1 records of
// rec_stride bytes, record 0 = the state on entry; a record holds the rows
// (x then z words of each slot), s0 and V[0..SF_DMAX) of W words, then d); a
// phase kernel evaluates every Clifford gate's phase factor at the fitting
// points from the records on both sides of it (one wavefront per pchunk
// consecutive gates) and adds it into its segment's sums (segacc: pe words
// per segment); a fit
// kernel turns each segment's sums into its program's phase E.
// ginfo[2 i] = segment of gate g0 + i, ginfo[2 i + 1] = index of its GF(2)
// Hadamard term in had (or -1).  In a dry run (no records) ginfo, if set,
// receives ginfo[i] = hull dimension on entry to terminal gate g0 + i.  rec == nullptr: everything in the track
// kernel.
struct TrackJob {
  TrackState* st;
  const DGate* gates;
  int32_t g0, g1;
  SegProg* prog;
  GF2Q* had;
  const uint8_t* outcomes;
  int32_t dry;
  int32_t nseg;            // segments of this range (split form)
  uint8_t* rec;
  int32_t* ginfo;
  uint32_t* segacc;
  int32_t rec_stride;      // bytes per record
  int32_t pe;              // words per segment in segacc (>= points of the largest d)
  int32_t pchunk;          // consecutive gates per phase-kernel wavefront
  int32_t pad2;
};

// longest gate range of one split-form track launch (bounds the records)
#define SF_RANGE_MAX 1024
// dry-run trace of a terminal gate: the hull dimension on entry, or'ed with
// this flag for a measurement whose cofactor adds a hull coordinate
#define SF_DTRACE_GROW 0x100

enum { TRK_OK = 0, TRK_E_DIM = 1, TRK_E_INTERNAL = 2, TRK_E_SEGS = 3 };

// Canonical view of a frame for readout: fully reduced row echelon form with
// rows sorted by pivot, the hull in that row order, and the echelon pivots of
// the hull's linear part (descending) whose bits rank the phase vectors.
struct ReadoutInfo {
  int32_t n, W, d, pad;
  int32_t piv[SF_DMAX];
  int32_t pad2[2];
  uint64_t s0[SF_WMAX];
  uint64_t V[SF_DMAX][SF_WMAX];
  uint64_t tab[SF_NMAX * 2 * SF_WMAX];
};

// One frame's element-kernel arguments in a batched round (one per frame,
// shared by every launch of the round).
struct ElemDesc {
  const SegProg* prog;     // the round's segment programs: segment k at prog + k
  const GF2Q* had;
  double2* amp;            // current amplitude buffer
  double2* amp_other;      // measurement filter target
  double2* partials;
  uint8_t* outcomes;
  double* pvals;
  double* scale;
  int* flags;
  uint64_t seed;
  const uint64_t* seedp;   // if set, the seed is read here (graph replays)
  int32_t G;
  int32_t nseg;            // segments of the frame's range this round
  int32_t mk;              // the measurement's program (prog + mk), or -1: none
  int32_t pad;
};

// Initialisation of one frame in a batched launch: basis words and seed are
// read from device memory (params[0..3] = basis, params[4] = seed).
struct InitDesc {
  TrackState* st;
  double2* amp;
  int* flags;
  const uint64_t* params;
  int32_t n, pad;
};
