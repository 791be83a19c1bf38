// Host side of libsframe.so: contexts, circuit loading, states, stepping and
// readout.  All frame arithmetic runs in the kernels of track.hip and
// elem.hip; this file validates arguments, owns device memory and queues
// launches on the context's stream.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/sframe.h"
#include "elem.hip"
#include "sf_dev.h"
#include "track.hip"

struct sf_ctx {
  int device;
  hipStream_t stream;
  sf_allocator alloc;
  int has_alloc;
  uint64_t budget, in_use;
  char err[512];
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct sf_circuit {
  sf_ctx* ctx;
  uint32_t n;
  std::vector<DGate> g;          // device gates (after rewriting)
  std::vector<size_t> orig_end;  // device index one past original gate i
  DevBuf dgates;
  int dmax;
  int max_segs, max_had;
  size_t n_meas;
  uint64_t projected;
};

struct sf_state {
  sf_ctx* ctx;
  const sf_circuit* c;
  DevBuf st, prog, had, amp[2], outcomes, pvals, scale, flags, partials, ri, count;
  int cur;
  size_t orig_done, dev_done, nmeas;
  uint64_t seed;
  int G;  // measurement reduction grid (fixed per state)
};

static sf_status fail(sf_ctx* ctx, sf_status st, const char* fmt, ...) {
  if (ctx) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(ctx->err, sizeof ctx->err, fmt, ap);
    va_end(ap);
  }
  return st;
}

#define HIPCHK(ctx, call)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(ctx, SF_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

static sf_status dalloc(sf_ctx* ctx, DevBuf* b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (ctx->budget && ctx->in_use + bytes > ctx->budget)
    return fail(ctx, SF_E_TOO_LARGE, "device budget exceeded (%llu + %zu > %llu bytes)",
                (unsigned long long)ctx->in_use, bytes, (unsigned long long)ctx->budget);
  void* p = nullptr;
  if (ctx->has_alloc) p = ctx->alloc.alloc(bytes, (void*)ctx->stream, ctx->alloc.user);
  else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
  if (!p) return fail(ctx, SF_E_OOM, "device allocation of %zu bytes failed", bytes);
  b->p = p;
  b->bytes = bytes;
  ctx->in_use += bytes;
  return SF_OK;
}

static void dfree(sf_ctx* ctx, DevBuf* b) {
  if (!b->p) return;
  if (ctx->has_alloc) ctx->alloc.free(b->p, b->bytes, (void*)ctx->stream, ctx->alloc.user);
  else hipFree(b->p);
  ctx->in_use -= b->bytes;
  b->p = nullptr;
  b->bytes = 0;
}

extern "C" sf_status sf_ctx_create(int device, void* hip_stream, const sf_allocator* alloc,
                                   uint64_t hbm_budget_bytes, sf_ctx** out) {
  if (!out) return SF_E_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return SF_E_DEVICE;
  if (device < 0 || device >= ndev) return SF_E_INVALID;
  if (hipSetDevice(device) != hipSuccess) return SF_E_DEVICE;
  sf_ctx* c = new (std::nothrow) sf_ctx();
  if (!c) return SF_E_OOM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->has_alloc = alloc && alloc->alloc && alloc->free;
  if (c->has_alloc) c->alloc = *alloc;
  c->budget = hbm_budget_bytes;
  c->in_use = 0;
  c->err[0] = 0;
  *out = c;
  return SF_OK;
}

extern "C" sf_status sf_ctx_destroy(sf_ctx* ctx) {
  delete ctx;
  return SF_OK;
}

extern "C" const char* sf_last_error(const sf_ctx* ctx) { return ctx ? ctx->err : "no context"; }

// ---------------------------------------------------------------------------
// Circuit loading
// ---------------------------------------------------------------------------
static DGate dg(int op, int q0, int q1 = 0) {
  DGate g;
  g.op = op; g.q0 = q0; g.q1 = q1; g.pad = 0; g.c = 1.0; g.s = 0.0;
  return g;
}

// diag(1, e^{i pi num/den}): multiples of pi/2 are Clifford (I, S, Z, S-dagger)
static void push_phase(std::vector<DGate>& v, int q, int64_t num, int64_t den) {
  if (den < 0) { num = -num; den = -den; }
  if ((2 * num) % den == 0) {
    int64_t m = ((2 * num) / den) % 4;
    if (m < 0) m += 4;
    if (m == 1) v.push_back(dg(DG_S, q));
    else if (m == 2) v.push_back(dg(DG_Z, q));
    else if (m == 3) v.push_back(dg(DG_SDG, q));
    return;
  }
  DGate g = dg(DG_NCPHASE, q);
  double th = M_PI * (double)num / (double)den;
  g.c = cos(th);
  g.s = sin(th);
  v.push_back(g);
}

static bool qok(uint32_t q, uint32_t n) { return q < n; }

extern "C" sf_status sf_circuit_load(sf_ctx* ctx, uint32_t n, const sf_gate* gates, size_t ng,
                                     sf_circuit** out) {
  if (!ctx || !out) return SF_E_INVALID;
  *out = nullptr;
  if (n < 1 || n > SF_NMAX) return fail(ctx, SF_E_INVALID, "qubit count %u outside 1..%d", n, SF_NMAX);
  if (ng && !gates) return fail(ctx, SF_E_INVALID, "null gate list");
  sf_circuit* c = new (std::nothrow) sf_circuit();
  if (!c) return fail(ctx, SF_E_OOM, "host allocation failed");
  c->ctx = ctx;
  c->n = n;
  c->n_meas = 0;
  for (size_t i = 0; i < ng; ++i) {
    const sf_gate& G = gates[i];
    auto bad = [&](const char* why) {
      delete c;
      return fail(ctx, SF_E_INVALID, "gate %zu (op %u): %s", i, G.op, why);
    };
    switch (G.op) {
      case SF_H: case SF_S: case SF_SDG: case SF_X: case SF_Y: case SF_Z:
        if (!qok(G.q0, n)) return bad("qubit out of range");
        c->g.push_back(dg((int)G.op, (int)G.q0));
        break;
      case SF_CNOT: case SF_CZ:
        if (!qok(G.q0, n) || !qok(G.q1, n)) return bad("qubit out of range");
        if (G.q0 == G.q1) return bad("control equals target");
        c->g.push_back(dg(G.op == SF_CNOT ? DG_CNOT : DG_CZ, (int)G.q0, (int)G.q1));
        break;
      case SF_T: case SF_TDG:
        if (!qok(G.q0, n)) return bad("qubit out of range");
        push_phase(c->g, (int)G.q0, G.op == SF_T ? 1 : -1, 4);
        break;
      case SF_PHASE:
        if (!qok(G.q0, n)) return bad("qubit out of range");
        if (G.theta_den == 0) return bad("zero angle denominator");
        push_phase(c->g, (int)G.q0, G.theta_num, G.theta_den);
        break;
      case SF_CPHASE: {
        if (!qok(G.q0, n) || !qok(G.q1, n)) return bad("qubit out of range");
        if (G.q0 == G.q1) return bad("control equals target");
        if (G.theta_den == 0) return bad("zero angle denominator");
        // theta c t = theta/2 (c + t - (c xor t))
        int cq = (int)G.q0, tq = (int)G.q1;
        push_phase(c->g, tq, G.theta_num, 2 * G.theta_den);
        c->g.push_back(dg(DG_CNOT, cq, tq));
        push_phase(c->g, tq, -G.theta_num, 2 * G.theta_den);
        c->g.push_back(dg(DG_CNOT, cq, tq));
        push_phase(c->g, cq, G.theta_num, 2 * G.theta_den);
        break;
      }
      case SF_TOF: {
        if (!qok(G.q0, n) || !qok(G.q1, n) || !qok(G.q2, n)) return bad("qubit out of range");
        if (G.q0 == G.q1 || G.q0 == G.q2 || G.q1 == G.q2) return bad("repeated qubit");
        int a = (int)G.q0, b = (int)G.q1, t = (int)G.q2;
        std::vector<DGate>& v = c->g;
        v.push_back(dg(DG_H, t));
        v.push_back(dg(DG_CNOT, b, t)); push_phase(v, t, -1, 4);
        v.push_back(dg(DG_CNOT, a, t)); push_phase(v, t, 1, 4);
        v.push_back(dg(DG_CNOT, b, t)); push_phase(v, t, -1, 4);
        v.push_back(dg(DG_CNOT, a, t)); push_phase(v, b, 1, 4); push_phase(v, t, 1, 4);
        v.push_back(dg(DG_H, t));
        v.push_back(dg(DG_CNOT, a, b)); push_phase(v, a, 1, 4); push_phase(v, b, -1, 4);
        v.push_back(dg(DG_CNOT, a, b));
        break;
      }
      case SF_MEASURE:
        if (!qok(G.q0, n)) return bad("qubit out of range");
        c->g.push_back(dg(DG_MEASURE, (int)G.q0));
        c->n_meas++;
        break;
      default:
        return bad("unknown operation");
    }
    c->orig_end.push_back(c->g.size());
  }
  // range planning: ranges end after each measurement
  c->max_segs = 1;
  c->max_had = 1;
  {
    int segs = 0, had = 0;
    bool open = false;
    for (size_t i = 0; i < c->g.size(); ++i) {
      int op = c->g[i].op;
      if (op == DG_H) ++had;
      if (op == DG_NCPHASE || op == DG_MEASURE) { ++segs; open = false; }
      else open = true;
      if (op == DG_MEASURE || i + 1 == c->g.size()) {
        int s = segs + (open ? 1 : 0);
        c->max_segs = std::max(c->max_segs, s);
        c->max_had = std::max(c->max_had, had);
        segs = 0; had = 0; open = false;
      }
    }
  }
  sf_status rc = dalloc(ctx, &c->dgates, sizeof(DGate) * std::max<size_t>(1, c->g.size()));
  if (rc != SF_OK) { delete c; return rc; }
  // dry run of the tableau track: frame bound of the whole circuit
  DevBuf dst;
  rc = dalloc(ctx, &dst, sizeof(TrackState));
  if (rc != SF_OK) { dfree(ctx, &c->dgates); delete c; return rc; }
  TrackState* h = (TrackState*)calloc(1, sizeof(TrackState));
  h->n = (int)n;
  h->W = (int)((n + 63) / 64);
  for (uint32_t q = 0; q < n; ++q) h->rz[q * SF_WMAX + (q >> 6)] = 1ull << (q & 63);
  hipError_t e = hipMemcpyAsync(dst.p, h, sizeof(TrackState), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && !c->g.empty())
    e = hipMemcpyAsync(c->dgates.p, c->g.data(), sizeof(DGate) * c->g.size(), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    TrackJob job;
    memset(&job, 0, sizeof job);
    job.st = (TrackState*)dst.p;
    job.gates = (const DGate*)c->dgates.p;
    job.g0 = 0;
    job.g1 = (int)c->g.size();
    job.dry = 1;
    hipLaunchKernelGGL(sf_track_kernel, dim3(1), dim3(TL), 0, ctx->stream, job, (const TrackJob*)nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h, dst.p, 64, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  int dmax = h->dmax, terr = h->error;
  free(h);
  dfree(ctx, &dst);
  if (e != hipSuccess) {
    dfree(ctx, &c->dgates);
    delete c;
    return fail(ctx, SF_E_DEVICE, "circuit analysis failed: %s", hipGetErrorString(e));
  }
  if (terr == TRK_E_DIM || dmax > SF_DMAX - 1) {
    dfree(ctx, &c->dgates);
    delete c;
    return fail(ctx, SF_E_TOO_LARGE, "frame bound 2^%d exceeds 2^%d", dmax, SF_DMAX - 1);
  }
  if (terr) {
    dfree(ctx, &c->dgates);
    delete c;
    return fail(ctx, SF_E_DEVICE, "tableau track reported internal error %d", terr);
  }
  c->dmax = dmax;
  uint64_t amp = (uint64_t)16 << dmax;
  c->projected = 2 * amp + sizeof(TrackState) + sizeof(ReadoutInfo) +
                 (uint64_t)c->max_segs * sizeof(SegProg) + (uint64_t)c->max_had * sizeof(GF2Q);
  *out = c;
  return SF_OK;
}

extern "C" sf_status sf_circuit_info(const sf_circuit* c, uint64_t* bound, uint64_t* bytes) {
  if (!c) return SF_E_INVALID;
  if (bound) *bound = (uint64_t)c->dmax;
  if (bytes) *bytes = c->projected;
  return SF_OK;
}

extern "C" sf_status sf_circuit_destroy(sf_circuit* c) {
  if (!c) return SF_OK;
  dfree(c->ctx, &c->dgates);
  delete c;
  return SF_OK;
}

// ---------------------------------------------------------------------------
// States
// ---------------------------------------------------------------------------
static void state_free(sf_state* s) {
  sf_ctx* ctx = s->ctx;
  DevBuf* all[] = {&s->st, &s->prog, &s->had, &s->amp[0], &s->amp[1], &s->outcomes, &s->pvals,
                   &s->scale, &s->flags, &s->partials, &s->ri, &s->count};
  for (DevBuf* b : all) dfree(ctx, b);
}

static int grid_for(int d) {
  uint64_t blocks = ((1ull << d) + EB - 1) / EB;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  return (int)blocks;
}

extern "C" sf_status sf_state_init(sf_ctx* ctx, const sf_circuit* c, const uint64_t* basis, uint64_t seed,
                                   sf_state** out) {
  if (!ctx || !c || !out) return SF_E_INVALID;
  *out = nullptr;
  sf_state* s = new (std::nothrow) sf_state();
  if (!s) return fail(ctx, SF_E_OOM, "host allocation failed");
  s->ctx = ctx;
  s->c = c;
  s->cur = 0;
  s->orig_done = s->dev_done = s->nmeas = 0;
  s->seed = seed;
  s->G = grid_for(c->dmax) > 1024 ? 1024 : grid_for(c->dmax);
  sf_status rc = SF_OK;
  size_t ampb = (size_t)16 << c->dmax;
  if ((rc = dalloc(ctx, &s->st, sizeof(TrackState))) ||
      (rc = dalloc(ctx, &s->prog, sizeof(SegProg) * (size_t)c->max_segs)) ||
      (rc = dalloc(ctx, &s->had, sizeof(GF2Q) * (size_t)c->max_had)) ||
      (rc = dalloc(ctx, &s->amp[0], ampb)) || (rc = dalloc(ctx, &s->amp[1], ampb)) ||
      (rc = dalloc(ctx, &s->outcomes, std::max<size_t>(1, c->n_meas))) ||
      (rc = dalloc(ctx, &s->pvals, 8 * std::max<size_t>(1, c->n_meas))) ||
      (rc = dalloc(ctx, &s->scale, 8)) || (rc = dalloc(ctx, &s->flags, 8)) ||
      (rc = dalloc(ctx, &s->partials, 16 * (size_t)s->G)) || (rc = dalloc(ctx, &s->ri, sizeof(ReadoutInfo))) ||
      (rc = dalloc(ctx, &s->count, 8))) {
    state_free(s);
    delete s;
    return rc;
  }
  TrackState* h = (TrackState*)calloc(1, sizeof(TrackState));
  h->n = (int)c->n;
  h->W = (int)((c->n + 63) / 64);
  for (uint32_t q = 0; q < c->n; ++q) h->rz[q * SF_WMAX + (q >> 6)] = 1ull << (q & 63);  // row q = Z_q
  if (basis)
    for (int w = 0; w < h->W; ++w) h->s0[w] = basis[w];
  if (c->n % 64) h->s0[h->W - 1] &= (1ull << (c->n % 64)) - 1ull;
  double one[2] = {1.0, 0.0};
  hipError_t e = hipMemcpyAsync(s->st.p, h, sizeof(TrackState), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s->amp[0].p, one, 16, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->flags.p, 0, 8, ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->outcomes.p, 0, std::max<size_t>(1, c->n_meas), ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);  // host buffers are on the stack
  free(h);
  if (e != hipSuccess) {
    state_free(s);
    delete s;
    return fail(ctx, SF_E_DEVICE, "state init: %s", hipGetErrorString(e));
  }
  *out = s;
  return SF_OK;
}

extern "C" sf_status sf_state_destroy(sf_state* s) {
  if (!s) return SF_OK;
  hipStreamSynchronize(s->ctx->stream);
  state_free(s);
  delete s;
  return SF_OK;
}

// Queue the device gates [a, b) (b ends at most right after a measurement).
static sf_status run_range(sf_state* s, size_t a, size_t b) {
  sf_ctx* ctx = s->ctx;
  const sf_circuit* c = s->c;
  if (a >= b) return SF_OK;
  TrackJob job;
  memset(&job, 0, sizeof job);
  job.st = (TrackState*)s->st.p;
  job.gates = (const DGate*)c->dgates.p;
  job.g0 = (int)a;
  job.g1 = (int)b;
  job.prog = (SegProg*)s->prog.p;
  job.had = (GF2Q*)s->had.p;
  job.outcomes = (const uint8_t*)s->outcomes.p;
  job.dry = 0;
  hipLaunchKernelGGL(sf_track_kernel, dim3(1), dim3(TL), 0, ctx->stream, job, (const TrackJob*)nullptr);
  HIPCHK(ctx, hipGetLastError());
  // segments: one per non-Clifford phase gate or measurement, plus a final one
  int nseg = 0;
  bool open = false, meas_last = false;
  for (size_t i = a; i < b; ++i) {
    int op = c->g[i].op;
    if (op == DG_NCPHASE || op == DG_MEASURE) { ++nseg; open = false; meas_last = op == DG_MEASURE; }
    else { open = true; meas_last = false; }
  }
  if (open) ++nseg;
  const int grid = grid_for(c->dmax);
  const SegProg* prog = (const SegProg*)s->prog.p;
  for (int k = 0; k < nseg; ++k) {
    hipLaunchKernelGGL(sf_seg_kernel, dim3(grid), dim3(EB), 0, ctx->stream, prog + k, (const GF2Q*)s->had.p,
                       (double2*)s->amp[s->cur].p);
  }
  if (meas_last) {
    const SegProg* sp = prog + (nseg - 1);
    hipLaunchKernelGGL(sf_meas_reduce, dim3(s->G), dim3(EB), 0, ctx->stream, sp, (const double2*)s->amp[s->cur].p,
                       (double2*)s->partials.p);
    hipLaunchKernelGGL(sf_meas_final, dim3(1), dim3(EB), 0, ctx->stream, sp, (const double2*)s->partials.p, s->G,
                       s->seed, (uint8_t*)s->outcomes.p, (double*)s->pvals.p, (double*)s->scale.p,
                       (int*)s->flags.p);
    hipLaunchKernelGGL(sf_meas_filter, dim3(grid), dim3(EB), 0, ctx->stream, sp, (const double2*)s->amp[s->cur].p,
                       (double2*)s->amp[s->cur ^ 1].p, (const uint8_t*)s->outcomes.p, (const double*)s->scale.p);
    s->cur ^= 1;
    s->nmeas++;
  }
  HIPCHK(ctx, hipGetLastError());
  return SF_OK;
}

extern "C" sf_status sf_step(sf_state* s, size_t max_gates, size_t* applied) {
  if (!s) return SF_E_INVALID;
  const sf_circuit* c = s->c;
  size_t o = s->orig_done, steps = 0;
  size_t a = s->dev_done, b = a;
  while (o < c->orig_end.size() && steps < max_gates) {
    size_t e = c->orig_end[o];
    bool meas = e > b && c->g[e - 1].op == DG_MEASURE;
    b = e;
    ++o;
    ++steps;
    if (meas) break;
  }
  sf_status rc = run_range(s, a, b);
  if (rc != SF_OK) return rc;
  s->orig_done = o;
  s->dev_done = b;
  if (applied) *applied = steps;
  return SF_OK;
}

extern "C" sf_status sf_run(sf_state* s) {
  if (!s) return SF_E_INVALID;
  size_t k = 1;
  while (k) {
    sf_status rc = sf_step(s, (size_t)-1, &k);
    if (rc != SF_OK) return rc;
  }
  return SF_OK;
}

static sf_status check_track(sf_state* s) {
  sf_ctx* ctx = s->ctx;
  int hdr[16];
  HIPCHK(ctx, hipMemcpyAsync(hdr, s->st.p, sizeof hdr, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  int terr = hdr[10];  // TrackState::error
  if (terr) return fail(ctx, SF_E_DEVICE, "tableau track reported error %d", terr);
  return SF_OK;
}

extern "C" sf_status sf_sync(sf_state* s) {
  if (!s) return SF_E_INVALID;
  HIPCHK(s->ctx, hipStreamSynchronize(s->ctx->stream));
  return check_track(s);
}

extern "C" sf_status sf_outcomes(sf_state* s, uint8_t* out, size_t cap, size_t* count) {
  if (!s) return SF_E_INVALID;
  sf_ctx* ctx = s->ctx;
  size_t m = std::min(cap, s->nmeas);
  if (m && out) HIPCHK(ctx, hipMemcpyAsync(out, s->outcomes.p, m, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (count) *count = s->nmeas;
  return check_track(s);
}

extern "C" sf_status sf_frame_size(sf_state* s, uint64_t* K) {
  if (!s || !K) return SF_E_INVALID;
  sf_ctx* ctx = s->ctx;
  HIPCHK(ctx, hipMemsetAsync(s->count.p, 0, 8, ctx->stream));
  hipLaunchKernelGGL(sf_count_kernel, dim3(grid_for(s->c->dmax)), dim3(EB), 0, ctx->stream,
                     (const TrackState*)s->st.p, (const double2*)s->amp[s->cur].p,
                     (unsigned long long*)s->count.p);
  HIPCHK(ctx, hipGetLastError());
  unsigned long long k = 0;
  HIPCHK(ctx, hipMemcpyAsync(&k, s->count.p, 8, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  *K = k;
  return check_track(s);
}

extern "C" sf_status sf_state_info(sf_state* s, size_t* done, int* fragile) {
  if (!s) return SF_E_INVALID;
  if (done) *done = s->orig_done;
  if (fragile) {
    int f = 0;
    HIPCHK(s->ctx, hipMemcpyAsync(&f, s->flags.p, 4, hipMemcpyDeviceToHost, s->ctx->stream));
    HIPCHK(s->ctx, hipStreamSynchronize(s->ctx->stream));
    *fragile = f;
  }
  return SF_OK;
}

extern "C" sf_status sf_read_frame(sf_state* s, uint64_t* tableau, uint64_t* sigma, double* amp, size_t cap,
                                   size_t* K_out) {
  if (!s) return SF_E_INVALID;
  sf_ctx* ctx = s->ctx;
  sf_status rc = check_track(s);
  if (rc != SF_OK) return rc;
  hipLaunchKernelGGL(sf_readout_track, dim3(1), dim3(TL), 0, ctx->stream, (const TrackState*)s->st.p,
                     (const uint8_t*)s->outcomes.p, (ReadoutInfo*)s->ri.p);
  HIPCHK(ctx, hipGetLastError());
  int hdr[4];
  HIPCHK(ctx, hipMemcpyAsync(hdr, s->ri.p, sizeof hdr, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  const int n = hdr[0], W = hdr[1], d = hdr[2];
  if (hdr[3]) return fail(ctx, SF_E_DEVICE, "hull basis lost rank");
  const uint64_t N = 1ull << d;
  const int nb = (int)((N + CH - 1) / CH);
  DevBuf tsig, flag, counts, total, osig, oamp;
  if ((rc = dalloc(ctx, &tsig, (size_t)N * W * 8)) || (rc = dalloc(ctx, &flag, (size_t)N)) ||
      (rc = dalloc(ctx, &counts, 4 * (size_t)nb)) || (rc = dalloc(ctx, &total, 8))) {
    dfree(ctx, &tsig); dfree(ctx, &flag); dfree(ctx, &counts); dfree(ctx, &total);
    return rc;
  }
  double2* tamp = (double2*)s->amp[s->cur ^ 1].p;
  const int grid = grid_for(d);
  hipLaunchKernelGGL(sf_readout_scatter, dim3(grid), dim3(EB), 0, ctx->stream, (const ReadoutInfo*)s->ri.p,
                     (const double2*)s->amp[s->cur].p, (uint64_t*)tsig.p, tamp, (uint8_t*)flag.p);
  hipLaunchKernelGGL(sf_compact_count, dim3(nb), dim3(EB), 0, ctx->stream, (const uint8_t*)flag.p, N,
                     (unsigned int*)counts.p);
  hipLaunchKernelGGL(sf_compact_scan, dim3(1), dim3(EB), 0, ctx->stream, (unsigned int*)counts.p, nb,
                     (unsigned long long*)total.p);
  unsigned long long K = 0;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&K, total.p, 8, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess && tableau) {
    std::vector<uint64_t> tab((size_t)n * 2 * W);
    e = hipMemcpy(tab.data(), (char*)s->ri.p + offsetof(ReadoutInfo, tab), tab.size() * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) memcpy(tableau, tab.data(), tab.size() * 8);
  }
  if (K_out) *K_out = (size_t)K;
  if (e == hipSuccess && K > cap) {
    dfree(ctx, &tsig); dfree(ctx, &flag); dfree(ctx, &counts); dfree(ctx, &total);
    return fail(ctx, SF_E_BUFSIZE, "frame has %llu elements, buffer holds %zu", K, cap);
  }
  if (e == hipSuccess && K > 0 && (sigma || amp)) {
    if ((rc = dalloc(ctx, &osig, (size_t)K * W * 8)) || (rc = dalloc(ctx, &oamp, (size_t)K * 16))) {
      dfree(ctx, &osig); dfree(ctx, &oamp);
      dfree(ctx, &tsig); dfree(ctx, &flag); dfree(ctx, &counts); dfree(ctx, &total);
      return rc;
    }
    hipLaunchKernelGGL(sf_compact_write, dim3(nb), dim3(EB), 0, ctx->stream, (const uint8_t*)flag.p,
                       (const uint64_t*)tsig.p, (const double2*)tamp, N, W, (const unsigned int*)counts.p,
                       (uint64_t*)osig.p, (double2*)oamp.p);
    e = hipGetLastError();
    if (e == hipSuccess && sigma) e = hipMemcpyAsync(sigma, osig.p, (size_t)K * W * 8, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess && amp) e = hipMemcpyAsync(amp, oamp.p, (size_t)K * 16, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  }
  dfree(ctx, &osig); dfree(ctx, &oamp);
  dfree(ctx, &tsig); dfree(ctx, &flag); dfree(ctx, &counts); dfree(ctx, &total);
  if (e != hipSuccess) return fail(ctx, SF_E_DEVICE, "readout: %s", hipGetErrorString(e));
  return SF_OK;
}
