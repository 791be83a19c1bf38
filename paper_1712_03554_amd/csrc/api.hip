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
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/sframe.h"
#include "elem.hip"
#include "sf_dev.h"
#include "track.hip"
#include "wide.hip"

enum { PK_TRACK = 0, PK_SEG, PK_MREDUCE, PK_MFINAL, PK_MFILTER, PK_READOUT, PK_INIT, PK_PHASE, PK_FIT, PK_WIDE, PK_N };

struct sf_ctx {
  int device;
  hipStream_t stream;
  sf_allocator alloc;
  int has_alloc;
  uint64_t budget, in_use;
  char err[512];
  // per-kernel timing with HIP events on the context stream: bit k of prof
  // enables kind k
  int prof, prof_open;
  std::vector<hipEvent_t> ev;   // pairs (start, end)
  std::vector<int> ev_kind;
  size_t ev_used;
  double prof_ms[PK_N];
  uint64_t prof_n[PK_N];
  // launch shape of the elementwise frame kernels (segment, measurement
  // filter) per hull dimension d: threads per block and blocks (grid-stride)
  int tune_block[SF_DMAX + 1], tune_grid[SF_DMAX + 1];
  // phase-kernel wavefronts per launch to aim for (each walks a chunk of
  // consecutive gates of one frame's range)
  int phase_waves;
  // second stream of sf_batch_run: the tableau tracks of round r + 1 run on
  // it while the phase and element kernels of round r run on `stream`
  // (default priority, non-blocking); nullptr: one stream only
  hipStream_t side = nullptr;
  hipEvent_t ev_track = nullptr, ev_meas = nullptr, ev_join = nullptr, ev_elem[2] = {nullptr, nullptr};
  hipStream_t prof_stream = nullptr;
  // pinned host chunks that stage batched-round descriptors for async copies;
  // reused after the stream has been synchronised
  std::vector<std::pair<char*, size_t>> pin;
  size_t pin_cur = 0, pin_off = 0;
};

// Pinned staging memory for an async host-to-device copy (nullptr if none
// can be had: the caller copies from pageable memory instead).
static void* pin_take(sf_ctx* ctx, size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  while (ctx->pin_cur < ctx->pin.size()) {
    auto& ch = ctx->pin[ctx->pin_cur];
    if (ctx->pin_off + bytes <= ch.second) {
      void* p = ch.first + ctx->pin_off;
      ctx->pin_off += bytes;
      return p;
    }
    ctx->pin_cur++;
    ctx->pin_off = 0;
  }
  const size_t sz = std::max<size_t>(bytes, (size_t)8 << 20);
  void* p = nullptr;
  if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess || !p) return nullptr;
  ctx->pin.push_back({(char*)p, sz});
  ctx->pin_cur = ctx->pin.size() - 1;
  ctx->pin_off = bytes;
  return p;
}

// after a stream synchronisation: every staged copy has completed
static void pin_release(sf_ctx* ctx) {
  ctx->pin_cur = 0;
  ctx->pin_off = 0;
}

// ---------------------------------------------------------------------------
// Allocation-free batched run.  The round descriptors (track jobs and element
// descriptors) and the error-gather table live in `scratch`, a file-scope
// device array of SF_SCRATCH_BYTES that every call on a device shares; its
// device address is looked up once per device at context creation
// (hipGetSymbolAddress) and only that address is used from the host.
// ---------------------------------------------------------------------------
#define SF_SCRATCH_BYTES ((size_t)8 << 20)
#define SF_MAX_DEVICES 64
static __device__ __align__(256) unsigned char scratch[SF_SCRATCH_BYTES];
static void* g_scratch_dev[SF_MAX_DEVICES];

static std::mutex g_scratch_mu;

// Once per device, with that device current (context creation).  A failed
// lookup leaves the address unset: sf_batch_run_noalloc then reports
// SF_E_DEVICE, every other call is unaffected.
static void scratch_lookup(int device) {
  if (device < 0 || device >= SF_MAX_DEVICES) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p) g_scratch_dev[device] = p;
}

// Circuits whose hull never exceeds this dimension (2^8 = EB slots, one
// reduction block) measure with one fused kernel per measurement.
#define SF_MSMALL_D 8
// Flattened batched element launches: slots per thread (segment launches and
// measurement filters, measured best apart), and at most this many blocks of
// EB threads per frame (a larger frame's threads stride over it).
#ifndef SF_BATCH_EPT_SEG
#define SF_BATCH_EPT_SEG 2
#endif
#ifndef SF_BATCH_EPT_FILTER
#define SF_BATCH_EPT_FILTER 8
#endif
#define SF_BATCH_BLOCKS_MAX 8192

// blocks of a frame whose hull dimension is at most d in a flattened launch
// with ept slots per thread
static uint32_t batch_blocks(int d, uint64_t cap, int ept) {
  if (d < 0) d = 0;
  if (d > SF_DMAX) d = SF_DMAX;
  const uint64_t per = (uint64_t)EB * (uint64_t)ept;
  const uint64_t nb = ((1ull << d) + per - 1) / per;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(nb, cap));
}

static int grid_for(int d) {
  uint64_t blocks = ((1ull << d) + EB - 1) / EB;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  return (int)blocks;
}

static int words_of(uint32_t n) { return (int)((n + 63) / 64); }

// Split form of the tableau track: always for frames of up to 128 qubits;
// for wider frames only in launches with at most SF_SPLIT_WIDE_MAX of them
// (with more the GPU is already full and the split costs more than it
// saves).  Bytes of one per-gate record and words of one segment's sums.
#define SF_SPLIT_WIDE_MAX 64
static bool split_form(uint32_t n) { return words_of(n) <= 2; }
static int rec_stride_of(uint32_t n) {
  const size_t W = (size_t)words_of(n);
  const size_t b = (size_t)n * 2 * W * 8 + (SF_DMAX + 1) * W * 8 + 8;
  return (int)((b + 255) & ~(size_t)255);
}
static int pe_of(int dmax) {
  const int d = dmax < 0 ? 0 : dmax;
  return (1 + d + d * (d - 1) / 2 + 3) & ~3;
}

static const void* phase_many_fn(int W) {
  switch (W) {
    case 1: return (const void*)sf_phase_many<1>;
    case 2: return (const void*)sf_phase_many<2>;
    case 3: return (const void*)sf_phase_many<3>;
    default: return (const void*)sf_phase_many<4>;
  }
}

static const void* track_many_fn(int W) {
  switch (W) {
    case 1: return (const void*)sf_track_many<1>;
    case 2: return (const void*)sf_track_many<2>;
    case 3: return (const void*)sf_track_many<3>;
    default: return (const void*)sf_track_many<4>;
  }
}

static void launch_track_one(hipStream_t st, const TrackJob& job, int W) {
  switch (W) {
    case 1: hipLaunchKernelGGL(sf_track_one<1>, dim3(1), dim3(TL), 0, st, job); break;
    case 2: hipLaunchKernelGGL(sf_track_one<2>, dim3(1), dim3(TL), 0, st, job); break;
    case 3: hipLaunchKernelGGL(sf_track_one<3>, dim3(1), dim3(TL), 0, st, job); break;
    default: hipLaunchKernelGGL(sf_track_one<4>, dim3(1), dim3(TL), 0, st, job); break;
  }
}

// Split form: the phase kernels of a track launch (len = longest range,
// nseg = most segments among the jobs).
static void launch_phase_one(sf_ctx* ctx, const TrackJob& job, int W);
static void launch_phase_many(sf_ctx* ctx, const TrackJob* jobs, int count, int W, int nchunk, int nseg,
                              size_t pad = 0);

// Phase-kernel launches that run beside the next round's tableau tracks take
// this much extra (unused) LDS per workgroup: fewer phase wavefronts per
// compute unit leave the tracks, which are on the critical path there, more
// of its issue slots and LDS bandwidth.  Alone, the phase kernel runs at its
// full occupancy.
#ifndef SF_PHASE_PAD_BESIDE
#define SF_PHASE_PAD_BESIDE 6144
#endif

static void launch_track_many(hipStream_t st, const TrackJob* jobs, int count, int W) {
  switch (W) {
    case 1: hipLaunchKernelGGL(sf_track_many<1>, dim3(count), dim3(TL), 0, st, jobs); break;
    case 2: hipLaunchKernelGGL(sf_track_many<2>, dim3(count), dim3(TL), 0, st, jobs); break;
    case 3: hipLaunchKernelGGL(sf_track_many<3>, dim3(count), dim3(TL), 0, st, jobs); break;
    default: hipLaunchKernelGGL(sf_track_many<4>, dim3(count), dim3(TL), 0, st, jobs); break;
  }
}

static void elem_shape(const sf_ctx* ctx, int d, int* block, int* grid) {
  if (d < 0) d = 0;
  if (d > SF_DMAX) d = SF_DMAX;
  *block = ctx->tune_block[d];
  *grid = ctx->tune_grid[d];
}

static void prof_begin(sf_ctx* ctx, int kind, hipStream_t on = nullptr) {
  ctx->prof_open = 0;
  ctx->prof_stream = on ? on : ctx->stream;
  if (!ctx->prof || !((ctx->prof >> kind) & 1)) return;
  size_t i = ctx->ev_used;
  if (2 * i + 2 > ctx->ev.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
    ctx->ev.push_back(a);
    ctx->ev.push_back(b);
    ctx->ev_kind.push_back(kind);
  }
  ctx->ev_kind[i] = kind;
  (void)hipEventRecord(ctx->ev[2 * i], ctx->prof_stream);
  ctx->prof_open = 1;
}

static void prof_end(sf_ctx* ctx) {
  if (!ctx->prof_open) return;
  (void)hipEventRecord(ctx->ev[2 * ctx->ev_used + 1], ctx->prof_stream);
  ctx->ev_used++;
  ctx->prof_open = 0;
}

static void prof_collect(sf_ctx* ctx) {
  for (size_t i = 0; i < ctx->ev_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev[2 * i], ctx->ev[2 * i + 1]) == hipSuccess) {
      ctx->prof_ms[ctx->ev_kind[i]] += ms;
      ctx->prof_n[ctx->ev_kind[i]] += 1;
    }
  }
  ctx->ev_used = 0;
}

// Phase-kernel wavefronts of a launch: about ctx->phase_waves, each walking
// pchunk consecutive gates (one gate per wavefront when frames are few).
// More and shorter chunks hide more latency but rebuild the record state at
// every chunk start; 65536 measured best on 1024 frames of 128 qubits
// (phase kernel 7.1 ms at 4096, 6.6 at 16384, 6.4 at 65536 per step).
#define SF_PHASE_WAVES 65536
static int phase_chunk(const sf_ctx* ctx, size_t total_gates) {
  const size_t w = (size_t)std::max(1, ctx->phase_waves);
  return (int)std::max<size_t>(1, (total_gates + w - 1) / w);
}

static void launch_phase_one(sf_ctx* ctx, const TrackJob& job, int W) {
  const int len = job.g1 - job.g0;
  if (job.dry || !job.rec || len <= 0) return;
  const int k = job.pchunk > 0 ? job.pchunk : 1;
  const int nchunk = (len + k - 1) / k;
  prof_begin(ctx, PK_PHASE);
  switch (W) {
    case 1: hipLaunchKernelGGL(sf_phase_one<1>, dim3(nchunk), dim3(TL), 0, ctx->stream, job); break;
    case 2: hipLaunchKernelGGL(sf_phase_one<2>, dim3(nchunk), dim3(TL), 0, ctx->stream, job); break;
    case 3: hipLaunchKernelGGL(sf_phase_one<3>, dim3(nchunk), dim3(TL), 0, ctx->stream, job); break;
    default: hipLaunchKernelGGL(sf_phase_one<4>, dim3(nchunk), dim3(TL), 0, ctx->stream, job); break;
  }
  prof_end(ctx);
  if (job.nseg > 0) {
    prof_begin(ctx, PK_FIT);
    hipLaunchKernelGGL(sf_fit_one, dim3(job.nseg), dim3(TL), 0, ctx->stream, job);
    prof_end(ctx);
  }
}

static void launch_phase_many(sf_ctx* ctx, const TrackJob* jobs, int count, int W, int nchunk, int nseg,
                              size_t pad) {
  if (count <= 0 || nchunk <= 0) return;
  prof_begin(ctx, PK_PHASE);
  const unsigned sh = (unsigned)pad;
  switch (W) {
    case 1: hipLaunchKernelGGL(sf_phase_many<1>, dim3(nchunk, count), dim3(TL), sh, ctx->stream, jobs); break;
    case 2: hipLaunchKernelGGL(sf_phase_many<2>, dim3(nchunk, count), dim3(TL), sh, ctx->stream, jobs); break;
    case 3: hipLaunchKernelGGL(sf_phase_many<3>, dim3(nchunk, count), dim3(TL), sh, ctx->stream, jobs); break;
    default: hipLaunchKernelGGL(sf_phase_many<4>, dim3(nchunk, count), dim3(TL), sh, ctx->stream, jobs); break;
  }
  prof_end(ctx);
  if (nseg > 0) {
    prof_begin(ctx, PK_FIT);
    hipLaunchKernelGGL(sf_fit_many, dim3(nseg, count), dim3(TL), 0, ctx->stream, jobs);
    prof_end(ctx);
  }
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct sf_circuit {
  sf_ctx* ctx;
  uint32_t n;
  // more than SF_NMAX qubits: a stabilizer circuit run by the wide-frame
  // kernels (one element, rows in device memory), without ranges or segments
  bool wide = false;
  std::vector<DGate> g;          // device gates (after rewriting)
  std::vector<size_t> orig_end;  // device index one past original gate i
  DevBuf dgates;
  int dmax;
  int max_segs, max_had;
  size_t n_meas;
  uint64_t projected;
  // every path ends a device range at these gate indices (original-gate
  // boundaries at most SF_RANGE_MAX gates apart), so that all paths split
  // the circuit into the same segments; rec_len = longest range
  std::vector<size_t> cuts;
  int rec_len;
  // the device ranges of a run from the first gate without a cap, planned
  // once at load (planning depends on the circuit only): rstart[dev index] =
  // the range starting there, or -1
  struct Range {
    size_t o0, a, b, o;
    int ns, ml, cl;  // segments, ends in a measurement, has a Clifford gate
    int dofs;        // its segments' hull dimensions at rdims[dofs..dofs + ns)
  };
  std::vector<Range> ranges;
  // hull dimension on entry to every terminal gate (device index; -1 for the
  // others), from the load-time dry run; per range, its segments' dimensions
  // (they size the element launches; the hull dimension does not depend on
  // measurement outcomes)
  std::vector<int8_t> dterm, rdims;
  // per gate: a measurement whose cofactor adds a hull coordinate (its
  // segment pass is folded into the measurement kernels)
  std::vector<uint8_t> mgrow;
  std::vector<int32_t> rstart;
};

static bool is_cut(const sf_circuit* c, size_t e) {
  return std::binary_search(c->cuts.begin(), c->cuts.end(), e);
}

static void build_range_table(sf_circuit* c);
static void fill_range_dims(sf_circuit* c);

struct sf_state {
  sf_ctx* ctx;
  const sf_circuit* c;
  DevBuf st, prog, had, amp[2], outcomes, pvals, scale, flags, partials, ri, count, adhoc;
  DevBuf rec, ginfo, segacc;  // split form of the tableau track
  DevBuf wbasis;              // wide frames: basis words for (re)initialisation
  // second set of the per-range buffers, for the odd rounds of an
  // overlapped sf_batch_run (allocated on first use)
  DevBuf prog2, had2, rec2, ginfo2, segacc2;
  int cur;
  size_t orig_done, dev_done, nmeas;
  size_t meas_cap;  // capacity of outcomes / pvals (circuit measurements, grown by sf_measure)
  int graph_refs;   // graphs that hold this state's buffers
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
  else (void)hipFree(b->p);
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
  // the tableau track keeps the tableau, its column-major copy and the hull
  // in LDS: it needs a device with more than 64 KiB per workgroup (gfx950)
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess ||
      lds < (int)(sizeof(TrackLdsProbe) + 1024))
    return SF_E_DEVICE;
  sf_ctx* c = new (std::nothrow) sf_ctx();
  if (!c) return SF_E_OOM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->has_alloc = alloc && alloc->alloc && alloc->free;
  if (c->has_alloc) c->alloc = *alloc;
  c->budget = hbm_budget_bytes;
  c->in_use = 0;
  c->err[0] = 0;
  c->prof = 0;
  c->prof_open = 0;
  c->ev_used = 0;
  for (int k = 0; k < PK_N; ++k) { c->prof_ms[k] = 0; c->prof_n[k] = 0; }
  for (int d = 0; d <= SF_DMAX; ++d) { c->tune_block[d] = EB; c->tune_grid[d] = grid_for(d); }
  c->phase_waves = SF_PHASE_WAVES;
  {
    hipStream_t side = nullptr;
    bool ok = hipStreamCreateWithFlags(&side, hipStreamNonBlocking) == hipSuccess;
    hipEvent_t* evs[5] = {&c->ev_track, &c->ev_meas, &c->ev_join, &c->ev_elem[0], &c->ev_elem[1]};
    for (hipEvent_t* e : evs) ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
    if (ok) {
      c->side = side;
    } else {
      for (hipEvent_t* e : evs)
        if (*e) { (void)hipEventDestroy(*e); *e = nullptr; }
      if (side) (void)hipStreamDestroy(side);
      (void)hipGetLastError();
    }
  }
  scratch_lookup(device);
  *out = c;
  return SF_OK;
}

extern "C" sf_status sf_ctx_destroy(sf_ctx* ctx) {
  if (!ctx) return SF_OK;
  (void)hipStreamSynchronize(ctx->stream);
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  for (auto& ch : ctx->pin) (void)hipHostFree(ch.first);
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    hipEvent_t evs[5] = {ctx->ev_track, ctx->ev_meas, ctx->ev_join, ctx->ev_elem[0], ctx->ev_elem[1]};
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(ctx->side);
  }
  delete ctx;
  return SF_OK;
}

extern "C" sf_status sf_profile(sf_ctx* ctx, int enable) {
  if (!ctx) return SF_E_INVALID;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  prof_collect(ctx);
  ctx->prof = enable;
  ctx->prof_open = 0;
  for (int k = 0; k < PK_N; ++k) { ctx->prof_ms[k] = 0; ctx->prof_n[k] = 0; }
  return SF_OK;
}

extern "C" sf_status sf_profile_read(sf_ctx* ctx, double* ms, uint64_t* launches, int nk) {
  if (!ctx) return SF_E_INVALID;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  prof_collect(ctx);
  for (int k = 0; k < nk && k < PK_N; ++k) {
    if (ms) ms[k] = ctx->prof_ms[k];
    if (launches) launches[k] = ctx->prof_n[k];
  }
  return SF_OK;
}

extern "C" const char* sf_last_error(const sf_ctx* ctx) { return ctx ? ctx->err : "no context"; }

// ---------------------------------------------------------------------------
// Circuit loading
// ---------------------------------------------------------------------------
// device gates that end a segment
static bool is_terminal(int op) { return op >= DG_NCPHASE; }

static DGate dg(int op, int q0, int q1 = 0) {
  DGate g;
  g.op = op; g.q0 = q0; g.q1 = q1; g.q2 = 0; g.c = 1.0; g.s = 0.0;
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
  if (n < 1 || n > SF_WIDE_NMAX) return fail(ctx, SF_E_INVALID, "qubit count %u outside 1..%d", n, SF_WIDE_NMAX);
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
      case SF_CPHASE_D: {
        if (!qok(G.q0, n) || !qok(G.q1, n)) return bad("qubit out of range");
        if (G.q0 == G.q1) return bad("control equals target");
        if (G.theta_den == 0) return bad("zero angle denominator");
        int64_t num = G.theta_num, den = G.theta_den;
        if (den < 0) { num = -num; den = -den; }
        if (num % den == 0) {  // theta a multiple of pi: identity or CZ
          if (((num / den) % 2 + 2) % 2) c->g.push_back(dg(DG_CZ, (int)G.q0, (int)G.q1));
          break;
        }
        // cofactor on both qubits (a split with phase 1), then the phase on
        // the elements where both read 1
        c->g.push_back(dg(DG_NCPHASE, (int)G.q0));
        c->g.push_back(dg(DG_NCPHASE, (int)G.q1));
        DGate g = dg(DG_CPH2, (int)G.q0, (int)G.q1);
        const double th = M_PI * (double)num / (double)den;
        g.c = cos(th);
        g.s = sin(th);
        c->g.push_back(g);
        break;
      }
      case SF_TOF_D: {
        if (!qok(G.q0, n) || !qok(G.q1, n) || !qok(G.q2, n)) return bad("qubit out of range");
        if (G.q0 == G.q1 || G.q0 == G.q2 || G.q1 == G.q2) return bad("repeated qubit");
        c->g.push_back(dg(DG_NCPHASE, (int)G.q0));
        c->g.push_back(dg(DG_NCPHASE, (int)G.q1));
        DGate g = dg(DG_CX2, (int)G.q0, (int)G.q1);
        g.q2 = (int)G.q2;
        c->g.push_back(g);
        break;
      }
      default:
        return bad("unknown operation");
    }
    c->orig_end.push_back(c->g.size());
  }
  if (n > SF_NMAX) {
    // wide frame: Clifford gates and measurements only
    for (size_t i = 0; i < c->g.size(); ++i)
      if (c->g[i].op >= DG_NCPHASE && c->g[i].op != DG_MEASURE) {
        delete c;
        return fail(ctx, SF_E_INVALID, "frames of more than %d qubits take stabilizer circuits only "
                    "(device gate %zu is not Clifford)", SF_NMAX, i);
      }
    c->wide = true;
    c->dmax = 0;
    c->max_segs = 1;
    c->max_had = 1;
    c->rec_len = 1;
    sf_status rc = dalloc(ctx, &c->dgates, sizeof(DGate) * std::max<size_t>(1, c->g.size()));
    hipError_t e = hipSuccess;
    if (rc == SF_OK && !c->g.empty())
      e = hipMemcpyAsync(c->dgates.p, c->g.data(), sizeof(DGate) * c->g.size(), hipMemcpyHostToDevice, ctx->stream);
    if (rc == SF_OK && e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (rc != SF_OK || e != hipSuccess) {
      dfree(ctx, &c->dgates);
      delete c;
      return rc != SF_OK ? rc : fail(ctx, SF_E_DEVICE, "gate upload: %s", hipGetErrorString(e));
    }
    const size_t W = words_of(n);
    c->projected = wide_layout((int)n).bytes + (4 * (size_t)n * W + W + 2) * 8 + 2 * c->n_meas * 9 + 64;
    *out = c;
    return SF_OK;
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
      if (is_terminal(op)) { ++segs; open = false; }
      else open = true;
      if (op == DG_MEASURE || i + 1 == c->g.size()) {
        int s = segs + (open ? 1 : 0);
        c->max_segs = std::max(c->max_segs, s);
        c->max_had = std::max(c->max_had, had);
        segs = 0; had = 0; open = false;
      }
    }
  }
  {
    size_t prev = 0, last = 0;
    for (size_t e : c->orig_end) {
      if (e - prev > SF_RANGE_MAX && last > prev) {
        c->cuts.push_back(last);
        prev = last;
      }
      last = e;
    }
    c->rec_len = (int)std::max<size_t>(1, std::min<size_t>(SF_RANGE_MAX, c->g.size()));
    // a cut can leave one more (open) segment in a range
    c->max_segs += 1;
  }
  build_range_table(c);
  sf_status rc = dalloc(ctx, &c->dgates, sizeof(DGate) * std::max<size_t>(1, c->g.size()));
  if (rc != SF_OK) { delete c; return rc; }
  // dry run of the tableau track: frame bound of the whole circuit, and the
  // hull dimension on entry to every terminal gate (in the gate-info slot,
  // which a dry run does not use otherwise)
  DevBuf dst, dtr;
  rc = dalloc(ctx, &dst, sizeof(TrackState));
  if (rc == SF_OK) rc = dalloc(ctx, &dtr, 4 * std::max<size_t>(1, c->g.size()));
  if (rc != SF_OK) { dfree(ctx, &dst); dfree(ctx, &c->dgates); delete c; return rc; }
  TrackState* h = (TrackState*)calloc(1, sizeof(TrackState));
  h->n = (int)n;
  h->W = (int)((n + 63) / 64);
  for (uint32_t q = 0; q < n; ++q) {
    h->rz[q * SF_WMAX + (q >> 6)] = 1ull << (q & 63);
    h->cz[q * SF_WMAX + (q >> 6)] = 1ull << (q & 63);
  }
  hipError_t e = hipMemcpyAsync(dst.p, h, sizeof(TrackState), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(dtr.p, 0xff, dtr.bytes, ctx->stream);
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
    job.ginfo = (int32_t*)dtr.p;
    launch_track_one(ctx->stream, job, words_of(n));
    e = hipGetLastError();
  }
  std::vector<int32_t> dtrace(std::max<size_t>(1, c->g.size()), -1);
  if (e == hipSuccess) e = hipMemcpyAsync(h, dst.p, 64, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dtrace.data(), dtr.p, 4 * dtrace.size(), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  int dmax = h->dmax, terr = h->error;
  free(h);
  dfree(ctx, &dst);
  dfree(ctx, &dtr);
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
  c->dterm.assign(c->g.size(), (int8_t)-1);
  c->mgrow.assign(c->g.size(), 0);
  for (size_t i = 0; i < c->g.size(); ++i) {
    if (!is_terminal(c->g[i].op)) continue;
    const int v = dtrace[i];
    c->dterm[i] = (int8_t)std::min(std::max(v < 0 ? -1 : (v & 0xff), -1), dmax);
    c->mgrow[i] = v >= 0 && (v & SF_DTRACE_GROW) && c->g[i].op == DG_MEASURE;
  }
  fill_range_dims(c);
  uint64_t amp = (uint64_t)16 << dmax;
  c->projected = 2 * amp + sizeof(TrackState) + sizeof(ReadoutInfo) +
                 (uint64_t)c->max_segs * sizeof(SegProg) + (uint64_t)c->max_had * sizeof(GF2Q);
  c->projected += (uint64_t)(c->rec_len + 1) * rec_stride_of(n) + (uint64_t)c->rec_len * 8 +
                  (uint64_t)c->max_segs * pe_of(dmax) * 4;
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
                   &s->scale, &s->flags, &s->partials, &s->ri, &s->count, &s->adhoc,
                   &s->rec, &s->ginfo, &s->segacc, &s->wbasis, &s->prog2, &s->had2, &s->rec2, &s->ginfo2,
                   &s->segacc2};
  for (DevBuf* b : all) dfree(ctx, b);
}

static sf_status queue_init(sf_state* s, const uint64_t* basis, uint64_t seed) {
  sf_ctx* ctx = s->ctx;
  if (s->c->wide) {
    const int n = (int)s->c->n, W = words_of(s->c->n);
    std::vector<uint64_t> b(W, 0);
    if (basis)
      for (int w = 0; w < W; ++w) b[w] = basis[w];
    s->cur = 0;
    s->orig_done = s->dev_done = s->nmeas = 0;
    s->seed = seed;
    HIPCHK(ctx, hipMemcpyAsync(s->wbasis.p, b.data(), W * 8, hipMemcpyHostToDevice, ctx->stream));
    prof_begin(ctx, PK_INIT);
    hipLaunchKernelGGL(sf_wide_init, dim3(1), dim3(WT), 0, ctx->stream, (unsigned char*)s->st.p, n,
                       (const uint64_t*)s->wbasis.p, seed, (int*)s->flags.p);
    prof_end(ctx);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SF_OK;
  }
  uint64_t b[4] = {0, 0, 0, 0};
  const int W = (int)((s->c->n + 63) / 64);
  if (basis)
    for (int w = 0; w < W; ++w) b[w] = basis[w];
  s->cur = 0;
  s->orig_done = s->dev_done = s->nmeas = 0;
  s->seed = seed;
  prof_begin(ctx, PK_INIT);
  hipLaunchKernelGGL(sf_init_state, dim3(1), dim3(EB), 0, ctx->stream, (TrackState*)s->st.p, (int)s->c->n, b[0],
                     b[1], b[2], b[3], (double2*)s->amp[0].p, (int*)s->flags.p);
  prof_end(ctx);
  HIPCHK(ctx, hipGetLastError());
  return SF_OK;
}

extern "C" sf_status sf_state_reset(sf_state* s, const uint64_t* basis, uint64_t seed) {
  if (!s) return SF_E_INVALID;
  return queue_init(s, basis, seed);
}

extern "C" sf_status sf_state_cycles(sf_state* s, uint64_t* cycles, int n) {
  if (!s || !cycles) return SF_E_INVALID;
  sf_ctx* ctx = s->ctx;
  if (s->c->wide) {
    for (int k = 0; k < n && k < 16; ++k) cycles[k] = 0;
    return SF_OK;
  }
  uint64_t c[16];
  HIPCHK(ctx, hipMemcpyAsync(c, (char*)s->st.p + offsetof(TrackState, cycles), sizeof c, hipMemcpyDeviceToHost,
                             ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < n && k < 16; ++k) cycles[k] = c[k];
  return SF_OK;
}

extern "C" sf_status sf_state_dim(sf_state* s, uint32_t* d) {
  if (!s || !d) return SF_E_INVALID;
  sf_ctx* ctx = s->ctx;
  if (s->c->wide) {
    *d = 0;
    return SF_OK;
  }
  int hdr[16];
  HIPCHK(ctx, hipMemcpyAsync(hdr, s->st.p, sizeof hdr, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  // d, pend, pend_r: a measurement's filter is applied to the hull lazily
  *d = (uint32_t)(hdr[2] - ((hdr[4] && hdr[8]) ? 1 : 0));
  return SF_OK;
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
  s->G = red_grid(c->dmax);  // partials of the largest reduction shape
  s->meas_cap = std::max<size_t>(1, c->n_meas);
  s->graph_refs = 0;
  sf_status rc = SF_OK;
  if (c->wide) {
    const size_t W = words_of(c->n);
    if ((rc = dalloc(ctx, &s->st, wide_layout((int)c->n).bytes)) ||
        (rc = dalloc(ctx, &s->outcomes, std::max<size_t>(1, c->n_meas))) ||
        (rc = dalloc(ctx, &s->pvals, 8 * std::max<size_t>(1, c->n_meas))) || (rc = dalloc(ctx, &s->flags, 8)) ||
        (rc = dalloc(ctx, &s->ri, (4 * (size_t)c->n * W + W + 2) * 8)) || (rc = dalloc(ctx, &s->wbasis, W * 8))) {
      state_free(s);
      delete s;
      return rc;
    }
    sf_status r2 = queue_init(s, basis, seed);
    if (r2 == SF_OK) {
      hipError_t e = hipMemsetAsync(s->outcomes.p, 0, std::max<size_t>(1, c->n_meas), ctx->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
      if (e != hipSuccess) r2 = fail(ctx, SF_E_DEVICE, "state init: %s", hipGetErrorString(e));
    }
    if (r2 != SF_OK) {
      state_free(s);
      delete s;
      return r2;
    }
    *out = s;
    return SF_OK;
  }
  size_t ampb = (size_t)16 << c->dmax;
  if ((rc = dalloc(ctx, &s->st, sizeof(TrackState))) ||
      (rc = dalloc(ctx, &s->prog, sizeof(SegProg) * (size_t)c->max_segs)) ||
      (rc = dalloc(ctx, &s->had, sizeof(GF2Q) * (size_t)c->max_had)) ||
      (rc = dalloc(ctx, &s->amp[0], ampb)) || (rc = dalloc(ctx, &s->amp[1], ampb)) ||
      (rc = dalloc(ctx, &s->outcomes, std::max<size_t>(1, c->n_meas))) ||
      (rc = dalloc(ctx, &s->pvals, 8 * std::max<size_t>(1, c->n_meas))) ||
      (rc = dalloc(ctx, &s->scale, 8)) || (rc = dalloc(ctx, &s->flags, 8)) ||
      (rc = dalloc(ctx, &s->partials, 16 * (size_t)s->G)) || (rc = dalloc(ctx, &s->ri, sizeof(ReadoutInfo))) ||
      (rc = dalloc(ctx, &s->count, 8)) ||
      (split_form(c->n) &&
       ((rc = dalloc(ctx, &s->rec, (size_t)(c->rec_len + 1) * rec_stride_of(c->n))) ||
        (rc = dalloc(ctx, &s->ginfo, (size_t)c->rec_len * 8)) ||
        (rc = dalloc(ctx, &s->segacc, (size_t)c->max_segs * pe_of(c->dmax) * 4))))) {
    state_free(s);
    delete s;
    return rc;
  }
  sf_status r2 = queue_init(s, basis, seed);
  if (r2 == SF_OK) {
    hipError_t e = hipMemsetAsync(s->outcomes.p, 0, std::max<size_t>(1, c->n_meas), ctx->stream);
    // gate info of the split form starts as "no segment, no Hadamard term"
    if (e == hipSuccess && s->ginfo.p) e = hipMemsetAsync(s->ginfo.p, 0xff, s->ginfo.bytes, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) r2 = fail(ctx, SF_E_DEVICE, "state init: %s", hipGetErrorString(e));
  }
  if (r2 != SF_OK) {
    state_free(s);
    delete s;
    return r2;
  }
  *out = s;
  return SF_OK;
}

extern "C" sf_status sf_state_destroy(sf_state* s) {
  if (!s) return SF_OK;
  if (s->graph_refs) return fail(s->ctx, SF_E_STATE, "state is part of a graph; destroy the graph first");
  (void)hipStreamSynchronize(s->ctx->stream);
  state_free(s);
  delete s;
  return SF_OK;
}

// Queue the device gates [a, b) of dgates (device copy) / hg (host copy); b
// ends at most right after a measurement.
// Record, gate-info and segment-sum buffers of a wide frame, allocated when a
// launch first runs it in split form (frames of up to 128 qubits get them at
// init).
// par: which of the two buffer sets (the second serves the odd rounds of an
// overlapped batched run); on: the stream that initialises the gate info.
static DevBuf& rec_buf(sf_state* s, int par) { return par ? s->rec2 : s->rec; }
static DevBuf& ginfo_buf(sf_state* s, int par) { return par ? s->ginfo2 : s->ginfo; }
static DevBuf& segacc_buf(sf_state* s, int par) { return par ? s->segacc2 : s->segacc; }
static const DevBuf& prog_buf(const sf_state* s, int par) { return par ? s->prog2 : s->prog; }
static const DevBuf& had_buf(const sf_state* s, int par) { return par ? s->had2 : s->had; }

static sf_status ensure_split_buffers(sf_state* s, int par = 0, hipStream_t on = nullptr) {
  DevBuf &rec = rec_buf(s, par), &ginfo = ginfo_buf(s, par), &segacc = segacc_buf(s, par);
  if (rec.p) return SF_OK;
  sf_ctx* ctx = s->ctx;
  const sf_circuit* c = s->c;
  sf_status rc;
  if ((rc = dalloc(ctx, &rec, (size_t)(c->rec_len + 1) * rec_stride_of(c->n))) ||
      (rc = dalloc(ctx, &ginfo, (size_t)c->rec_len * 8)) ||
      (rc = dalloc(ctx, &segacc, (size_t)c->max_segs * pe_of(c->dmax) * 4))) {
    dfree(ctx, &rec);
    dfree(ctx, &ginfo);
    dfree(ctx, &segacc);
    return rc;
  }
  HIPCHK(ctx, hipMemsetAsync(ginfo.p, 0xff, ginfo.bytes, on ? on : ctx->stream));
  return SF_OK;
}

// Programs and Hadamard terms of the second set.
static sf_status ensure_second_set(sf_state* s) {
  if (s->prog2.p) return SF_OK;
  sf_status rc;
  if ((rc = dalloc(s->ctx, &s->prog2, s->prog.bytes)) || (rc = dalloc(s->ctx, &s->had2, s->had.bytes))) {
    dfree(s->ctx, &s->prog2);
    dfree(s->ctx, &s->had2);
    return rc;
  }
  return SF_OK;
}

// The split-form buffers of a state in a track job (use: this launch runs the
// frame in split form).
static void split_fields(sf_state* s, TrackJob* job, int nseg, bool use = true, int par = 0) {
  job->nseg = nseg;
  if (!use || !rec_buf(s, par).p || job->dry) return;
  job->rec = (uint8_t*)rec_buf(s, par).p;
  job->ginfo = (int32_t*)ginfo_buf(s, par).p;
  job->segacc = (uint32_t*)segacc_buf(s, par).p;
  job->rec_stride = rec_stride_of(s->c->n);
  job->pe = pe_of(s->c->dmax);
  job->pchunk = 1;
}

// The device range ending before gate b ends in a measurement whose segment
// pass is folded into the measurement kernels (no launch needed for it).
static bool folded_meas(const sf_circuit* c, size_t b) {
  return b > 0 && b - 1 < c->mgrow.size() && c->mgrow[b - 1];
}

static sf_status run_chunk(sf_state* s, const DGate* dgates, const DGate* hg, size_t a, size_t b) {
  sf_ctx* ctx = s->ctx;
  const sf_circuit* c = s->c;
  if (a >= b) return SF_OK;
  size_t nm = 0;
  for (size_t i = a; i < b; ++i) nm += hg[i].op == DG_MEASURE;
  if (s->nmeas + nm > s->meas_cap)
    return fail(ctx, SF_E_STATE, "outcome buffer holds %zu measurements, %zu needed", s->meas_cap, s->nmeas + nm);
  // segments: one per non-Clifford phase gate or measurement, plus a final one
  int nseg = 0;
  bool open = false, meas_last = false;
  for (size_t i = a; i < b; ++i) {
    int op = hg[i].op;
    if (is_terminal(op)) { ++nseg; open = false; meas_last = op == DG_MEASURE; }
    else { open = true; meas_last = false; }
  }
  if (open) ++nseg;
  if (c->wide) {
    WideJob job;
    memset(&job, 0, sizeof job);
    job.base = (unsigned char*)s->st.p;
    job.gates = dgates;
    job.g0 = (int)a;
    job.g1 = (int)b;
    job.outcomes = (uint8_t*)s->outcomes.p;
    job.pvals = (double*)s->pvals.p;
    job.flags = (int*)s->flags.p;
    prof_begin(ctx, PK_WIDE);
    hipLaunchKernelGGL(sf_wide_one, dim3(1), dim3(WT), 0, ctx->stream, job);
    prof_end(ctx);
    HIPCHK(ctx, hipGetLastError());
    s->nmeas += nm;
    return SF_OK;
  }
  if (nseg > c->max_segs || b - a > (size_t)c->rec_len)
    return fail(ctx, SF_E_STATE, "range of %zu gates with %d segments exceeds the state's buffers", b - a, nseg);
  // one frame: the split form pays for every width
  sf_status rs = ensure_split_buffers(s);
  if (rs != SF_OK) return rs;
  TrackJob job;
  memset(&job, 0, sizeof job);
  job.st = (TrackState*)s->st.p;
  job.gates = dgates;
  job.g0 = (int)a;
  job.g1 = (int)b;
  job.prog = (SegProg*)s->prog.p;
  job.had = (GF2Q*)s->had.p;
  job.outcomes = (const uint8_t*)s->outcomes.p;
  job.dry = 0;
  split_fields(s, &job, nseg);
  prof_begin(ctx, PK_TRACK);
  launch_track_one(ctx->stream, job, words_of(c->n));
  prof_end(ctx);
  // (a range without Clifford gates keeps the zero phase the track wrote)
  bool anycliff = false;
  for (size_t i = a; i < b && !anycliff; ++i) anycliff = hg[i].op < DG_NCPHASE;
  if (anycliff) launch_phase_one(ctx, job, words_of(c->n));
  HIPCHK(ctx, hipGetLastError());
  int eb, grid;
  elem_shape(ctx, c->dmax, &eb, &grid);
  const SegProg* prog = (const SegProg*)s->prog.p;
  if (c->dmax <= SF_MSMALL_D) {
    // small frame: the range's segments and its measurement in one block
    prof_begin(ctx, PK_SEG);
    hipLaunchKernelGGL(sf_elem_small, dim3(1), dim3(EB), 0, ctx->stream, (const SegProg*)prog, nseg,
                       (const GF2Q*)s->had.p, (double2*)s->amp[s->cur].p, (double2*)s->amp[s->cur ^ 1].p,
                       meas_last ? 1 : 0, s->seed, (uint8_t*)s->outcomes.p, (double*)s->pvals.p,
                       (double*)s->scale.p, (int*)s->flags.p);
    prof_end(ctx);
    if (meas_last) {
      s->cur ^= 1;
      s->nmeas++;
    }
    HIPCHK(ctx, hipGetLastError());
    return SF_OK;
  }
  const int kseg = (meas_last && dgates == (const DGate*)c->dgates.p && folded_meas(c, b)) ? nseg - 1 : nseg;
  for (int k = 0; k < kseg; ++k) {
    prof_begin(ctx, PK_SEG);
    hipLaunchKernelGGL(sf_seg_kernel, dim3(grid), dim3(eb), 0, ctx->stream, prog + k, (const GF2Q*)s->had.p,
                       (double2*)s->amp[s->cur].p);
    prof_end(ctx);
  }
  if (meas_last) {
    const SegProg* sp = prog + (nseg - 1);
    prof_begin(ctx, PK_MREDUCE);
    hipLaunchKernelGGL(sf_meas_reduce, dim3(s->G), dim3(EB), 0, ctx->stream, sp, (const GF2Q*)s->had.p,
                       (const double2*)s->amp[s->cur].p, (double2*)s->partials.p);
    prof_end(ctx);
    prof_begin(ctx, PK_MFILTER);
    hipLaunchKernelGGL(sf_meas_filter, dim3(grid), dim3(eb), 0, ctx->stream, sp, (const GF2Q*)s->had.p,
                       (const double2*)s->partials.p,
                       s->seed, (uint8_t*)s->outcomes.p, (double*)s->pvals.p, (double*)s->scale.p,
                       (int*)s->flags.p, (const double2*)s->amp[s->cur].p, (double2*)s->amp[s->cur ^ 1].p);
    prof_end(ctx);
    s->cur ^= 1;
    s->nmeas++;
  }
  HIPCHK(ctx, hipGetLastError());
  return SF_OK;
}

// Device gates [a, b): in ranges that end at the circuit's cuts (the
// circuit's own gates) so that every path forms the same segments.
static sf_status run_gates(sf_state* s, const DGate* dgates, const DGate* hg, size_t a, size_t b) {
  const sf_circuit* c = s->c;
  if (dgates == (const DGate*)c->dgates.p) {
    auto it = std::upper_bound(c->cuts.begin(), c->cuts.end(), a);
    for (; it != c->cuts.end() && *it < b; ++it) {
      sf_status rc = run_chunk(s, dgates, hg, a, *it);
      if (rc != SF_OK) return rc;
      a = *it;
    }
  }
  return run_chunk(s, dgates, hg, a, b);
}

static sf_status run_range(sf_state* s, size_t a, size_t b) {
  return run_gates(s, (const DGate*)s->c->dgates.p, s->c->g.data(), a, b);
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

static sf_status check_track(sf_state* s);

// Ad-hoc measurement of qubit q between circuit gates.  The frame bound of
// the rest of the circuit is re-derived first (the tableau track does not
// depend on outcomes, so a dry pass from the current tableau gives it); a
// measurement that would let a later gate outgrow the state's buffers is
// refused and leaves the state as it was.
extern "C" sf_status sf_measure(sf_state* s, uint32_t q, int* outcome) {
  if (!s) return SF_E_INVALID;
  sf_ctx* ctx = s->ctx;
  const sf_circuit* c = s->c;
  if (q >= c->n) return fail(ctx, SF_E_INVALID, "qubit %u out of range (n = %u)", q, c->n);
  sf_status rc = check_track(s);
  if (rc != SF_OK) return rc;
  if (!s->adhoc.p && (rc = dalloc(ctx, &s->adhoc, sizeof(DGate)))) return rc;
  DGate g;
  memset(&g, 0, sizeof g);
  g.op = DG_MEASURE;
  g.q0 = (int)q;
  HIPCHK(ctx, hipMemcpyAsync(s->adhoc.p, &g, sizeof g, hipMemcpyHostToDevice, ctx->stream));
  hipError_t e = hipSuccess;
  if (!c->wide) {
  // dry pass: this measurement, then the rest of the circuit
  DevBuf tmp;
  if ((rc = dalloc(ctx, &tmp, sizeof(TrackState)))) return rc;
  e = hipMemcpyAsync(tmp.p, s->st.p, sizeof(TrackState), hipMemcpyDeviceToDevice, ctx->stream);
  for (int part = 0; part < 2 && e == hipSuccess; ++part) {
    TrackJob job;
    memset(&job, 0, sizeof job);
    job.st = (TrackState*)tmp.p;
    job.gates = part == 0 ? (const DGate*)s->adhoc.p : (const DGate*)c->dgates.p;
    job.g0 = part == 0 ? 0 : (int)s->dev_done;
    job.g1 = part == 0 ? 1 : (int)c->g.size();
    job.dry = 1;
    if (job.g0 >= job.g1) break;
    launch_track_one(ctx->stream, job, words_of(c->n));
    e = hipGetLastError();
  }
  int hdr[16];
  if (e == hipSuccess) e = hipMemcpyAsync(hdr, tmp.p, sizeof hdr, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dfree(ctx, &tmp);
  if (e != hipSuccess) return fail(ctx, SF_E_DEVICE, "measure: %s", hipGetErrorString(e));
  static_assert(offsetof(TrackState, dmax) == 9 * 4 && offsetof(TrackState, error) == 10 * 4, "header layout");
  const int dmax_after = hdr[9], terr = hdr[10];
  if (terr == TRK_E_DIM || dmax_after > c->dmax)
    return fail(ctx, SF_E_TOO_LARGE, "after measuring qubit %u the rest of the circuit needs 2^%d elements, "
                "the state holds 2^%d", q, dmax_after, c->dmax);
  if (terr) return fail(ctx, SF_E_DEVICE, "tableau track reported internal error %d", terr);
  }
  // room for this outcome and for those of the circuit's remaining
  // measurements, whose indices it shifts by one
  size_t rem = 0;
  for (size_t i = s->dev_done; i < c->g.size(); ++i) rem += c->g[i].op == DG_MEASURE;
  const size_t need = s->nmeas + 1 + rem;
  if (need > s->meas_cap) {
    if (s->graph_refs) return fail(ctx, SF_E_STATE, "measurement buffers of a state in a graph cannot grow");
    size_t cap = std::max<size_t>(2 * s->meas_cap, need);
    DevBuf no, np;
    if ((rc = dalloc(ctx, &no, cap))) return rc;
    if ((rc = dalloc(ctx, &np, 8 * cap))) { dfree(ctx, &no); return rc; }
    e = hipMemsetAsync(no.p, 0, cap, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(no.p, s->outcomes.p, s->meas_cap, hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(np.p, s->pvals.p, 8 * s->meas_cap, hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) { dfree(ctx, &no); dfree(ctx, &np); return fail(ctx, SF_E_DEVICE, "measure: %s", hipGetErrorString(e)); }
    dfree(ctx, &s->outcomes);
    dfree(ctx, &s->pvals);
    s->outcomes = no;
    s->pvals = np;
    s->meas_cap = cap;
  }
  const size_t idx = s->nmeas;
  if ((rc = run_gates(s, (const DGate*)s->adhoc.p, &g, 0, 1))) return rc;
  uint8_t o = 0;
  HIPCHK(ctx, hipMemcpyAsync(&o, (const uint8_t*)s->outcomes.p + idx, 1, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if ((rc = check_track(s))) return rc;
  if (outcome) *outcome = o;
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
  if (s->c->wide) {
    *K = 1;
    return check_track(s);
  }
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
  if (s->c->wide) {
    const size_t n = s->c->n, W = words_of(s->c->n);
    uint64_t* out = (uint64_t*)s->ri.p;
    prof_begin(ctx, PK_READOUT);
    hipLaunchKernelGGL(sf_wide_readout, dim3(1), dim3(WT), 0, ctx->stream, (const unsigned char*)s->st.p, out,
                       out + n * 2 * W + W + 2);
    prof_end(ctx);
    HIPCHK(ctx, hipGetLastError());
    std::vector<uint64_t> h(n * 2 * W + W + 2);
    HIPCHK(ctx, hipMemcpyAsync(h.data(), out, h.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (K_out) *K_out = 1;
    if (tableau && cap >= 1) memcpy(tableau, h.data(), n * 2 * W * 8);
    if (cap < 1) return fail(ctx, SF_E_BUFSIZE, "frame has 1 element, buffer holds 0");
    if (sigma) memcpy(sigma, h.data() + n * 2 * W, W * 8);
    if (amp) memcpy(amp, h.data() + n * 2 * W + W, 16);
    return SF_OK;
  }
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
  if (e == hipSuccess && tableau && K <= cap) {
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

// ---------------------------------------------------------------------------
// Batched execution: every round runs, for each unfinished frame, the gates up
// to and including its next measurement.  The tableau tracks of all frames
// share one launch (one wavefront each); the element kernels of segment k of
// every frame share one launch (grid y = frame).
// ---------------------------------------------------------------------------
// Host bookkeeping of a frame's progress through its circuit.
struct Progress {
  size_t orig_done, dev_done, nmeas;
  int cur;
};

static Progress progress_of(const sf_state* s) { return Progress{s->orig_done, s->dev_done, s->nmeas, s->cur}; }

static void set_progress(sf_state* s, const Progress& p) {
  s->orig_done = p.orig_done;
  s->dev_done = p.dev_done;
  s->nmeas = p.nmeas;
  s->cur = p.cur;
}

// The range runs to the next measurement; with cap > 0 it may also stop right
// after its cap-th non-Clifford phase gate when that gate ends a circuit gate
// (a segment boundary either way, so the segments and their arithmetic are
// those of the uncapped run).
static void plan_range(const sf_circuit* c, const Progress& pr, size_t* a, size_t* b, size_t* orig_after, int* nseg,
                       int* meas_last, int cap = 0, int* has_cliff = nullptr) {
  if (cap == 0 && pr.dev_done < c->rstart.size()) {
    const int k = c->rstart[pr.dev_done];
    if (k >= 0 && c->ranges[(size_t)k].o0 == pr.orig_done) {
      const sf_circuit::Range& r = c->ranges[(size_t)k];
      *a = r.a;
      *b = r.b;
      *orig_after = r.o;
      *nseg = r.ns;
      *meas_last = r.ml;
      if (has_cliff) *has_cliff = r.cl;
      return;
    }
  }
  size_t o = pr.orig_done, e = pr.dev_done;
  *a = pr.dev_done;
  int terms = 0;
  while (o < c->orig_end.size()) {
    size_t end = c->orig_end[o];
    for (size_t i = e; i < end; ++i) terms += is_terminal(c->g[i].op) && c->g[i].op != DG_MEASURE;
    bool meas = end > e && c->g[end - 1].op == DG_MEASURE;
    bool cut = cap > 0 && terms >= cap && end > e && is_terminal(c->g[end - 1].op);
    e = end;
    ++o;
    if (meas || cut || is_cut(c, e)) break;
  }
  *b = e;
  *orig_after = o;
  int ns = 0;
  bool open = false, ml = false, cl = false;
  for (size_t i = *a; i < *b; ++i) {
    int op = c->g[i].op;
    if (is_terminal(op)) { ++ns; open = false; ml = op == DG_MEASURE; }
    else { open = true; ml = false; cl = true; }
  }
  if (open) ++ns;
  *nseg = ns;
  *meas_last = ml ? 1 : 0;
  if (has_cliff) *has_cliff = cl ? 1 : 0;
}

// Plans the uncapped ranges of a run from the first gate once (the walk of
// plan_range for every range start of that run).
static void build_range_table(sf_circuit* c) {
  c->ranges.clear();
  c->rstart.assign(c->g.size() + 1, -1);
  Progress p{0, 0, 0, 0};
  while (p.orig_done < c->orig_end.size()) {
    sf_circuit::Range r;
    r.o0 = p.orig_done;
    r.dofs = -1;
    plan_range(c, p, &r.a, &r.b, &r.o, &r.ns, &r.ml, 0, &r.cl);
    if (r.b <= r.a && r.o <= r.o0) break;  // no progress: leave the rest to the walk
    c->rstart[r.a] = (int32_t)c->ranges.size();
    c->ranges.push_back(r);
    p.orig_done = r.o;
    p.dev_done = r.b;
  }
}

// Per range, the hull dimension of each segment: a segment ending in a
// terminal gate runs at the dimension on entry to it; an open segment at the
// end of a range at the dimension on entry to the next terminal gate (its
// continuation), or the circuit's bound.
static void fill_range_dims(sf_circuit* c) {
  c->rdims.clear();
  const size_t G = c->g.size();
  std::vector<int8_t> next(G + 1, (int8_t)c->dmax);
  for (size_t i = G; i-- > 0;) next[i] = c->dterm[i] >= 0 ? c->dterm[i] : next[i + 1];
  for (sf_circuit::Range& r : c->ranges) {
    r.dofs = (int)c->rdims.size();
    bool open = false;
    int k = 0;
    for (size_t i = r.a; i < r.b; ++i) {
      if (is_terminal(c->g[i].op)) {
        c->rdims.push_back(c->dterm[i] >= 0 ? c->dterm[i] : (int8_t)c->dmax);
        open = false;
        ++k;
      } else {
        open = true;
      }
    }
    if (open) { c->rdims.push_back(next[r.b]); ++k; }
    if (k != r.ns) {  // inconsistent: size by the bound
      c->rdims.resize(r.dofs);
      r.dofs = -1;
    }
  }
}

static ElemDesc elem_desc(const sf_state* s, int cur, const SegProg* prog, const uint64_t* seedp, int par = 0) {
  ElemDesc e;
  memset(&e, 0, sizeof e);
  e.prog = prog;
  e.had = (const GF2Q*)had_buf(s, par).p;
  e.amp = (double2*)s->amp[cur].p;
  e.amp_other = (double2*)s->amp[cur ^ 1].p;
  e.partials = (double2*)s->partials.p;
  e.outcomes = (uint8_t*)s->outcomes.p;
  e.pvals = (double*)s->pvals.p;
  e.scale = (double*)s->scale.p;
  e.flags = (int*)s->flags.p;
  e.seed = s->seed;
  e.seedp = seedp;
  e.G = s->G;
  return e;
}

// One batched round: the track job of every frame with work left and the
// element descriptors (one per frame: its programs, buffers and the number
// of its segments this round, and its measurement's program if the range
// ends in one).
struct RoundPlan {
  std::vector<TrackJob> jobs;
  std::vector<ElemDesc> desc;
  int na = 0, kmax = 0;
  bool anym = false;
  bool msmall = false;  // every frame's hull stays within SF_MSMALL_D: fused measurement kernel
  int wcount[SF_WMAX + 1] = {0, 0, 0, 0, 0};  // frames per word count (jobs are ordered by it)
  int wlen[SF_WMAX + 1] = {0, 0, 0, 0, 0};    // per word count: longest range, most segments,
  int wseg[SF_WMAX + 1] = {0, 0, 0, 0, 0};    // phase-kernel chunks of the longest range
  int wchunk[SF_WMAX + 1] = {0, 0, 0, 0, 0};  // 0: no Clifford gate in the group's ranges
  // block starts of the flattened element launches: rows 0..kmax-1 the
  // segments, row kmax the measurement reductions, row kmax+1 the
  // measurement filters; na + 1 entries per row (the last is the row's grid)
  std::vector<uint32_t> bst;
  // the bytes copied to the device: desc, then bst at offset bst_off
  size_t bst_off = 0;
  std::vector<char> dbytes;
};

static unsigned row_blocks(const RoundPlan& rp, int r) { return rp.bst[(size_t)r * (rp.na + 1) + rp.na]; }

// row r's block starts in the device copy whose descriptors are at dd
static const uint32_t* row_starts(const RoundPlan& rp, const ElemDesc* dd, int r) {
  return (const uint32_t*)((const char*)dd + rp.bst_off) + (size_t)r * (rp.na + 1);
}

// Plans the next round from the progress pr[] and advances it; false when no
// frame has work left or on an error (*err set; *bad = index of the state
// that caused it, or -1).  seedp[i] (optional) is where frame i's seed is
// read.  Nothing is queued before an error.
// With noalloc, a wide frame whose record buffers are not allocated yet runs
// with the in-kernel phase evaluation instead of allocating them.
static bool plan_round(sf_state* const* states, size_t ns, Progress* pr, int cap, const uint64_t* const* seedp,
                       RoundPlan* rp, sf_status* err, int* bad = nullptr, bool noalloc = false, int par = 0,
                       hipStream_t on = nullptr) {
  std::vector<int> act;
  std::vector<size_t> A(ns), B(ns), O(ns);
  std::vector<int> NS(ns), ML(ns), CL(ns);
  *err = SF_OK;
  if (bad) *bad = -1;
  for (size_t i = 0; i < ns; ++i) {
    const sf_circuit* c = states[i]->c;
    if (pr[i].orig_done >= c->orig_end.size()) continue;
    plan_range(c, pr[i], &A[i], &B[i], &O[i], &NS[i], &ML[i], cap, &CL[i]);
    if (ML[i] && pr[i].nmeas + 1 > states[i]->meas_cap) {
      *err = fail(states[i]->ctx, SF_E_STATE, "state %zu: outcome buffer holds %zu measurements", i,
                  states[i]->meas_cap);
      if (bad) *bad = (int)i;
      return false;
    }
    act.push_back((int)i);
  }
  if (act.empty()) return false;
  // one track launch per word count: order the frames by it (a stable
  // counting sort over the word counts)
  for (int w = 0; w <= SF_WMAX; ++w) rp->wcount[w] = rp->wlen[w] = rp->wseg[w] = rp->wchunk[w] = 0;
  {
    std::vector<int> wof(act.size());
    for (size_t t = 0; t < act.size(); ++t) {
      wof[t] = words_of(states[act[t]]->c->n);
      rp->wcount[wof[t]]++;
    }
    int start[SF_WMAX + 2] = {0};
    for (int w = 0; w <= SF_WMAX; ++w) start[w + 1] = start[w] + rp->wcount[w];
    std::vector<int> sorted(act.size());
    for (size_t t = 0; t < act.size(); ++t) sorted[start[wof[t]]++] = act[t];
    act.swap(sorted);
  }
  const int na = (int)act.size();
  rp->na = na;
  rp->jobs.assign(na, TrackJob{});
  rp->kmax = 0;
  rp->anym = false;
  int dm = 0;
  for (int j = 0; j < na; ++j) {
    const int i = act[j];
    sf_state* s = states[i];
    TrackJob& jb = rp->jobs[j];
    memset(&jb, 0, sizeof jb);
    jb.st = (TrackState*)s->st.p;
    jb.gates = (const DGate*)s->c->dgates.p;
    jb.g0 = (int)A[i];
    jb.g1 = (int)B[i];
    jb.prog = (SegProg*)prog_buf(s, par).p;
    jb.had = (GF2Q*)had_buf(s, par).p;
    jb.outcomes = (const uint8_t*)s->outcomes.p;
    if (NS[i] > s->c->max_segs || B[i] - A[i] > (size_t)s->c->rec_len) {
      *err = fail(s->ctx, SF_E_STATE, "state %d: range of %zu gates with %d segments exceeds its buffers", i,
                  B[i] - A[i], NS[i]);
      if (bad) *bad = i;
      return false;
    }
    const bool use = (split_form(s->c->n) || rp->wcount[words_of(s->c->n)] <= SF_SPLIT_WIDE_MAX) &&
                     (!noalloc || s->rec.p);
    if (use && (*err = ensure_split_buffers(s, par, on)) != SF_OK) {
      if (bad) *bad = i;
      return false;
    }
    split_fields(s, &jb, NS[i], use, par);
    const int wi = words_of(s->c->n);
    rp->wlen[wi] = std::max(rp->wlen[wi], (int)(B[i] - A[i]));
    rp->wseg[wi] = std::max(rp->wseg[wi], NS[i]);
    rp->kmax = std::max(rp->kmax, NS[i]);
    dm = std::max(dm, s->c->dmax);
    rp->anym |= ML[i] != 0;
  }
  // phase-kernel chunk per word count: the group's gates over SF_PHASE_WAVES
  {
    // (jobs are ordered by word count: job j's count follows from the counts)
    std::vector<int> jw(na);
    for (int w = 0, j = 0; w <= SF_WMAX; ++w)
      for (int t = 0; t < rp->wcount[w]; ++t) jw[j++] = w;
    size_t gates[SF_WMAX + 1] = {0, 0, 0, 0, 0};
    bool cliff[SF_WMAX + 1] = {false, false, false, false, false};
    for (int j = 0; j < na; ++j) {
      const TrackJob& jb = rp->jobs[j];
      if (jb.rec) gates[jw[j]] += (size_t)(jb.g1 - jb.g0);
      cliff[jw[j]] = cliff[jw[j]] || CL[act[j]] != 0;
    }
    int kw[SF_WMAX + 1];
    for (int w = 0; w <= SF_WMAX; ++w) {
      kw[w] = phase_chunk(states[act[0]]->ctx, gates[w]);
      rp->wchunk[w] = (rp->wlen[w] > 0 && cliff[w] && gates[w] > 0) ? (rp->wlen[w] + kw[w] - 1) / kw[w] : 0;
    }
    for (int j = 0; j < na; ++j)
      if (rp->jobs[j].rec) rp->jobs[j].pchunk = kw[jw[j]];
  }
  rp->msmall = dm <= SF_MSMALL_D;
  // flattened element launches: in row k (segment k; then the measurements'
  // reduction row and filter row) frame j takes its own number of blocks,
  // from the bound on its hull dimension there, so small frames beside a
  // large one start no idle blocks.  Row r holds na + 1 block starts.
  {
    const int R = rp->kmax + 2;
    const size_t stride = (size_t)na + 1;
    rp->bst.assign((size_t)R * stride, 0);
    // every row's total stays a valid grid size
    const uint64_t bcap = std::min<uint64_t>(SF_BATCH_BLOCKS_MAX, (uint64_t)INT32_MAX / (uint64_t)na);
    for (int j = 0; j < na; ++j) {
      const int i = act[j];
      const sf_circuit* c = states[i]->c;
      const int8_t* dims = nullptr;
      if (cap == 0 && A[i] < c->rstart.size()) {
        const int r = c->rstart[A[i]];
        if (r >= 0 && c->ranges[(size_t)r].o0 == pr[i].orig_done && c->ranges[(size_t)r].dofs >= 0 &&
            c->ranges[(size_t)r].ns == NS[i])
          dims = c->rdims.data() + c->ranges[(size_t)r].dofs;
      }
      const int kseg = (ML[i] && folded_meas(c, B[i])) ? NS[i] - 1 : NS[i];
      for (int k = 0; k < kseg; ++k)
        rp->bst[(size_t)k * stride + j + 1] = batch_blocks(dims ? (int)dims[k] : c->dmax, bcap, SF_BATCH_EPT_SEG);
      if (ML[i] && NS[i] > 0) {
        const int dl = dims ? std::min((int)dims[NS[i] - 1] + 1, c->dmax) : c->dmax;
        rp->bst[(size_t)rp->kmax * stride + j + 1] = (uint32_t)red_grid(dl);
        rp->bst[(size_t)(rp->kmax + 1) * stride + j + 1] = batch_blocks(dl, bcap, SF_BATCH_EPT_FILTER);
      }
    }
    for (int r = 0; r < R; ++r) {
      uint64_t sum = 0;
      for (int j = 0; j < na; ++j) {
        sum += rp->bst[(size_t)r * stride + j + 1];
        if (sum > (uint64_t)INT32_MAX) {
          *err = fail(states[act[0]]->ctx, SF_E_TOO_LARGE, "%d frames need more than 2^31 blocks in one launch", na);
          return false;
        }
        rp->bst[(size_t)r * stride + j + 1] = (uint32_t)sum;
      }
    }
  }
  // one descriptor per frame, shared by every launch of the round
  rp->desc.resize((size_t)na);
  for (int j = 0; j < na; ++j) {
    const int i = act[j];
    sf_state* s = states[i];
    ElemDesc& e = rp->desc[(size_t)j];
    e = elem_desc(s, pr[i].cur, (const SegProg*)prog_buf(s, par).p, seedp ? seedp[i] : nullptr, par);
    e.nseg = NS[i];
    e.mk = (ML[i] && NS[i] > 0) ? NS[i] - 1 : -1;
  }
  rp->bst_off = (rp->desc.size() * sizeof(ElemDesc) + 255) & ~(size_t)255;
  rp->dbytes.assign(rp->bst_off + rp->bst.size() * sizeof(uint32_t), 0);
  memcpy(rp->dbytes.data(), rp->desc.data(), rp->desc.size() * sizeof(ElemDesc));
  memcpy(rp->dbytes.data() + rp->bst_off, rp->bst.data(), rp->bst.size() * sizeof(uint32_t));
  for (int j = 0; j < na; ++j) {
    const int i = act[j];
    pr[i].dev_done = B[i];
    pr[i].orig_done = O[i];
    if (ML[i]) { pr[i].cur ^= 1; pr[i].nmeas++; }
  }
  return true;
}

// Device descriptor buffers of batched rounds and the host copies they were
// filled from (kept alive until the stream is synchronised).
struct BatchScratch {
  DevBuf djobs, ddesc;
  std::vector<std::vector<TrackJob>> keep_jobs;
  std::vector<std::vector<char>> keep_desc;
};

// jobs then (at a 256-byte boundary) descriptors: one copy per round
static size_t desc_offset(size_t job_bytes) { return (job_bytes + 255) & ~(size_t)255; }

// device bytes of a round's descriptors and block starts (RoundPlan::dbytes)
// for ns frames of at most maxseg segments
static size_t desc_capacity(size_t ns, int maxseg) {
  ns = std::max<size_t>(1, ns);
  return desc_offset(ns * sizeof(ElemDesc)) + (size_t)(maxseg + 2) * (ns + 1) * sizeof(uint32_t);
}

static sf_status scratch_reserve(sf_ctx* ctx, BatchScratch* bs, size_t ns, int maxseg) {
  size_t need_d = desc_capacity(ns, maxseg);
  size_t need_j = desc_offset(std::max<size_t>(1, ns) * sizeof(TrackJob)) + need_d;
  sf_status rc;
  if (bs->djobs.bytes < need_j) {
    dfree(ctx, &bs->djobs);
    if ((rc = dalloc(ctx, &bs->djobs, need_j))) return rc;
  }
  if (bs->ddesc.bytes < need_d) {
    dfree(ctx, &bs->ddesc);
    if ((rc = dalloc(ctx, &bs->ddesc, need_d))) return rc;
  }
  return SF_OK;
}

static void scratch_free(sf_ctx* ctx, BatchScratch* bs) {
  dfree(ctx, &bs->djobs);
  dfree(ctx, &bs->ddesc);
  bs->keep_jobs.clear();
  bs->keep_desc.clear();
}

// The measurement coin in a kernel of its own (once per frame) when the
// filter launch has many blocks: each block of the fused filter kernel sums
// the reduction's partials again, which costs more than a launch there.
#define SF_COIN_APART_BLOCKS 2048
static bool coin_apart(const RoundPlan& rp) { return row_blocks(rp, rp.kmax + 1) > SF_COIN_APART_BLOCKS; }

// Kernel launches of one planned round, with its descriptors at djobs/ddesc.
static void launch_round(sf_ctx* ctx, const RoundPlan& rp, const TrackJob* djobs, const ElemDesc* dd) {
  const int na = rp.na;
  int off = 0;
  for (int w = 1; w <= SF_WMAX; ++w) {
    if (!rp.wcount[w]) continue;
    prof_begin(ctx, PK_TRACK);
    launch_track_many(ctx->stream, djobs + off, rp.wcount[w], w);
    prof_end(ctx);
    launch_phase_many(ctx, djobs + off, rp.wcount[w], w, rp.wchunk[w], rp.wseg[w]);
    off += rp.wcount[w];
  }
  if (rp.msmall) {
    // small frames: each frame's segments and measurement in one block
    if (rp.kmax > 0 || rp.anym) {
      prof_begin(ctx, PK_SEG);
      hipLaunchKernelGGL(sf_elem_small_batch, dim3(na), dim3(EB), 0, ctx->stream, dd, rp.kmax, na,
                         rp.anym ? 1 : 0);
      prof_end(ctx);
    }
    return;
  }
  for (int k = 0; k < rp.kmax; ++k) {
    if (!row_blocks(rp, k)) continue;
    prof_begin(ctx, PK_SEG);
    hipLaunchKernelGGL(sf_seg_batch, dim3(row_blocks(rp, k)), dim3(EB), 0, ctx->stream, dd, row_starts(rp, dd, k),
                       na, k);
    prof_end(ctx);
  }
  if (rp.anym) {
    const ElemDesc* dm = dd;
    const uint32_t* rb = row_starts(rp, dd, rp.kmax);
    const uint32_t* fb = row_starts(rp, dd, rp.kmax + 1);
    const dim3 rg(row_blocks(rp, rp.kmax)), fg(row_blocks(rp, rp.kmax + 1));
    prof_begin(ctx, PK_MREDUCE);
    hipLaunchKernelGGL(sf_meas_reduce_batch, rg, dim3(EB), 0, ctx->stream, dm, rb, na);
    prof_end(ctx);
    if (coin_apart(rp)) {
      prof_begin(ctx, PK_MFINAL);
      hipLaunchKernelGGL(sf_meas_coin_batch, dim3(na), dim3(EB), 0, ctx->stream, dm);
      prof_end(ctx);
      prof_begin(ctx, PK_MFILTER);
      hipLaunchKernelGGL(sf_meas_apply_batch, fg, dim3(EB), 0, ctx->stream, dm, fb, na);
      prof_end(ctx);
    } else {
      prof_begin(ctx, PK_MFILTER);
      hipLaunchKernelGGL(sf_meas_filter_batch, fg, dim3(EB), 0, ctx->stream, dm, fb, na);
      prof_end(ctx);
    }
  }
}

// Queue one round for the given states: each unfinished state runs its gates
// up to and including its next measurement (or its cap-th non-Clifford phase
// gate).  *active = number of states that had work.  Asynchronous; the
// scratch must be large enough.
// staged: the descriptors go through pinned memory (the caller synchronises
// the stream and releases it before the next batch).
// *bad (optional) receives the index of the state that made planning fail
// (nothing was queued then), or -1.
static sf_status batch_round(sf_ctx* ctx, sf_state* const* states, size_t ns, BatchScratch* bs, int* active,
                             int cap = 0, bool staged = false, int* bad = nullptr, bool noalloc = false) {
  std::vector<Progress> pr(ns);
  for (size_t i = 0; i < ns; ++i) pr[i] = progress_of(states[i]);
  RoundPlan rp;
  sf_status err;
  *active = 0;
  if (!plan_round(states, ns, pr.data(), cap, nullptr, &rp, &err, bad, noalloc)) return err;
  *active = rp.na;
  if (staged) {
    const size_t bj = rp.na * sizeof(TrackJob), bd = rp.dbytes.size();
    const size_t offd = desc_offset(bj);
    char* h = offd + bd <= bs->djobs.bytes ? (char*)pin_take(ctx, offd + bd) : nullptr;
    if (h) {
      memcpy(h, rp.jobs.data(), bj);
      memcpy(h + offd, rp.dbytes.data(), bd);
      HIPCHK(ctx, hipMemcpyAsync(bs->djobs.p, h, offd + bd, hipMemcpyHostToDevice, ctx->stream));
      launch_round(ctx, rp, (const TrackJob*)bs->djobs.p, (const ElemDesc*)((char*)bs->djobs.p + offd));
      HIPCHK(ctx, hipGetLastError());
      for (size_t i = 0; i < ns; ++i) set_progress(states[i], pr[i]);
      return SF_OK;
    }
  }
  const size_t ndesc = rp.dbytes.size();
  bs->keep_jobs.push_back(std::move(rp.jobs));
  bs->keep_desc.push_back(std::move(rp.dbytes));
  HIPCHK(ctx, hipMemcpyAsync(bs->djobs.p, bs->keep_jobs.back().data(), rp.na * sizeof(TrackJob),
                             hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(bs->ddesc.p, bs->keep_desc.back().data(), ndesc, hipMemcpyHostToDevice, ctx->stream));
  launch_round(ctx, rp, (const TrackJob*)bs->djobs.p, (const ElemDesc*)bs->ddesc.p);
  HIPCHK(ctx, hipGetLastError());
  for (size_t i = 0; i < ns; ++i) set_progress(states[i], pr[i]);
  return SF_OK;
}

// One round of an overlapped batched run (round index r, buffer set r & 1):
// the descriptors and the tableau tracks go to the side stream, the phase,
// fit, segment and measurement kernels to the context's stream after the
// tracks.  The tracks of the next round can then run while this round's
// other kernels do: a track reads the previous round's measurement outcomes
// (it waits for them when that round measured) and writes the per-range
// buffers of its set (it waits until the round two back, the last one that
// used them, has finished on the context's stream).
static sf_status batch_round_ov(sf_ctx* ctx, sf_state* const* states, size_t ns, BatchScratch* bsets, int* active,
                                int round, bool* prev_meas) {
  const int par = round & 1;
  hipStream_t T = ctx->side, E = ctx->stream;
  std::vector<Progress> pr(ns);
  for (size_t i = 0; i < ns; ++i) pr[i] = progress_of(states[i]);
  RoundPlan rp;
  sf_status err;
  *active = 0;
  if (!plan_round(states, ns, pr.data(), 0, nullptr, &rp, &err, nullptr, false, par, T)) return err;
  *active = rp.na;
  BatchScratch* bs = &bsets[par];
  if (round >= 2) HIPCHK(ctx, hipStreamWaitEvent(T, ctx->ev_elem[par], 0));
  if (*prev_meas) HIPCHK(ctx, hipStreamWaitEvent(T, ctx->ev_meas, 0));
  const size_t bj = rp.na * sizeof(TrackJob), bd = rp.dbytes.size();
  const size_t offd = desc_offset(bj);
  const TrackJob* djobs;
  const ElemDesc* dd;
  char* h = offd + bd <= bs->djobs.bytes ? (char*)pin_take(ctx, offd + bd) : nullptr;
  if (h) {
    memcpy(h, rp.jobs.data(), bj);
    memcpy(h + offd, rp.dbytes.data(), bd);
    HIPCHK(ctx, hipMemcpyAsync(bs->djobs.p, h, offd + bd, hipMemcpyHostToDevice, T));
    djobs = (const TrackJob*)bs->djobs.p;
    dd = (const ElemDesc*)((char*)bs->djobs.p + offd);
  } else {
    bs->keep_jobs.push_back(std::move(rp.jobs));
    bs->keep_desc.push_back(std::move(rp.dbytes));
    HIPCHK(ctx, hipMemcpyAsync(bs->djobs.p, bs->keep_jobs.back().data(), bj, hipMemcpyHostToDevice, T));
    HIPCHK(ctx, hipMemcpyAsync(bs->ddesc.p, bs->keep_desc.back().data(), bd, hipMemcpyHostToDevice, T));
    djobs = (const TrackJob*)bs->djobs.p;
    dd = (const ElemDesc*)bs->ddesc.p;
  }
  int off = 0;
  for (int w = 1; w <= SF_WMAX; ++w) {
    if (!rp.wcount[w]) continue;
    prof_begin(ctx, PK_TRACK, T);
    launch_track_many(T, djobs + off, rp.wcount[w], w);
    prof_end(ctx);
    off += rp.wcount[w];
  }
  HIPCHK(ctx, hipEventRecord(ctx->ev_track, T));
  HIPCHK(ctx, hipStreamWaitEvent(E, ctx->ev_track, 0));
  RoundPlan el = rp;          // the element part of launch_round, without the tracks
  for (int w = 0; w <= SF_WMAX; ++w) el.wcount[w] = 0;
  off = 0;
  // without a measurement in this round the next round's tracks need not
  // wait for it: they run beside this round's phase kernels
  const size_t pad = rp.anym ? 0 : SF_PHASE_PAD_BESIDE;
  for (int w = 1; w <= SF_WMAX; ++w) {
    if (!rp.wcount[w]) continue;
    launch_phase_many(ctx, djobs + off, rp.wcount[w], w, rp.wchunk[w], rp.wseg[w], pad);
    off += rp.wcount[w];
  }
  launch_round(ctx, el, djobs, dd);
  HIPCHK(ctx, hipGetLastError());
  if (rp.anym) HIPCHK(ctx, hipEventRecord(ctx->ev_meas, E));
  HIPCHK(ctx, hipEventRecord(ctx->ev_elem[par], E));
  *prev_meas = rp.anym;
  for (size_t i = 0; i < ns; ++i) set_progress(states[i], pr[i]);
  return SF_OK;
}

// Device memory of check_tracks' gather launch for ns states.
static size_t gather_bytes(size_t ns) { return ((ns * sizeof(void*) + 255) & ~(size_t)255) + ns * sizeof(int); }

// Device-side errors of many states with one gather launch and one copy.
// work: device memory of gather_bytes(ns) bytes, or nullptr to allocate it.
static sf_status check_tracks(sf_ctx* ctx, sf_state* const* states, size_t ns, void* work = nullptr) {
  if (ns == 0) return SF_OK;
  if (ns == 1) return check_track(states[0]);
  DevBuf buf;
  const size_t off = (ns * sizeof(void*) + 255) & ~(size_t)255;
  if (work) {
    buf.p = work;
  } else {
    sf_status rc = dalloc(ctx, &buf, gather_bytes(ns));
    if (rc) return rc;
  }
  std::vector<const TrackState*> ptr(ns);
  for (size_t i = 0; i < ns; ++i) ptr[i] = (const TrackState*)states[i]->st.p;
  std::vector<int> errs(ns, 0);
  hipError_t e = hipMemcpyAsync(buf.p, ptr.data(), ns * sizeof(void*), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    const int grid = (int)std::min<size_t>(1024, (ns + EB - 1) / EB);
    hipLaunchKernelGGL(sf_gather_errors, dim3(grid), dim3(EB), 0, ctx->stream, (const TrackState* const*)buf.p,
                       (int)ns, (int*)((char*)buf.p + off));
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(errs.data(), (char*)buf.p + off, ns * sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (!work) dfree(ctx, &buf);
  if (e != hipSuccess) return fail(ctx, SF_E_DEVICE, "error check: %s", hipGetErrorString(e));
  for (size_t i = 0; i < ns; ++i)
    if (errs[i]) return fail(ctx, SF_E_DEVICE, "state %zu: tableau track reported error %d", i, errs[i]);
  return SF_OK;
}

// Wide frames of a batch: the rest of each circuit, one workgroup per frame in
// one launch.
static sf_status run_wide_batch(sf_ctx* ctx, const std::vector<sf_state*>& ws, DevBuf* djobs) {
  if (ws.empty()) return SF_OK;
  std::vector<WideJob> jobs(ws.size());
  std::vector<size_t> nm(ws.size(), 0);
  for (size_t i = 0; i < ws.size(); ++i) {
    sf_state* s = ws[i];
    const sf_circuit* c = s->c;
    for (size_t g = s->dev_done; g < c->g.size(); ++g) nm[i] += c->g[g].op == DG_MEASURE;
    if (s->nmeas + nm[i] > s->meas_cap)
      return fail(ctx, SF_E_STATE, "outcome buffer holds %zu measurements, %zu needed", s->meas_cap, s->nmeas + nm[i]);
    WideJob& j = jobs[i];
    memset(&j, 0, sizeof j);
    j.base = (unsigned char*)s->st.p;
    j.gates = (const DGate*)c->dgates.p;
    j.g0 = (int)s->dev_done;
    j.g1 = (int)c->g.size();
    j.outcomes = (uint8_t*)s->outcomes.p;
    j.pvals = (double*)s->pvals.p;
    j.flags = (int*)s->flags.p;
  }
  sf_status rc = dalloc(ctx, djobs, jobs.size() * sizeof(WideJob));
  if (rc != SF_OK) return rc;
  HIPCHK(ctx, hipMemcpyAsync(djobs->p, jobs.data(), jobs.size() * sizeof(WideJob), hipMemcpyHostToDevice, ctx->stream));
  prof_begin(ctx, PK_WIDE);
  hipLaunchKernelGGL(sf_wide_run, dim3((unsigned)jobs.size()), dim3(WT), 0, ctx->stream, (const WideJob*)djobs->p);
  prof_end(ctx);
  HIPCHK(ctx, hipGetLastError());
  for (size_t i = 0; i < ws.size(); ++i) {
    sf_state* s = ws[i];
    s->nmeas += nm[i];
    s->orig_done = s->c->orig_end.size();
    s->dev_done = s->c->g.size();
  }
  return SF_OK;
}

static bool any_wide(sf_state* const* states, size_t ns) {
  for (size_t i = 0; i < ns; ++i)
    if (states[i] && states[i]->c->wide) return true;
  return false;
}

extern "C" sf_status sf_batch_run(sf_ctx* ctx, sf_state* const* all, size_t ns_all) {
  if (!ctx || (ns_all && !all)) return SF_E_INVALID;
  int maxseg = 1;
  std::vector<sf_state*> reg, wsts;
  for (size_t i = 0; i < ns_all; ++i) {
    if (!all[i] || all[i]->ctx != ctx) return fail(ctx, SF_E_INVALID, "state %zu is not of this context", i);
    (all[i]->c->wide ? wsts : reg).push_back(all[i]);
    if (!all[i]->c->wide) maxseg = std::max(maxseg, all[i]->c->max_segs);
  }
  if (ns_all == 0) return SF_OK;
  DevBuf wj;
  sf_status wrc = run_wide_batch(ctx, wsts, &wj);
  if (wrc != SF_OK) {
    (void)hipStreamSynchronize(ctx->stream);
    dfree(ctx, &wj);
    return wrc;
  }
  if (reg.empty()) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    dfree(ctx, &wj);
    if (e != hipSuccess) return fail(ctx, SF_E_DEVICE, "batch run: %s", hipGetErrorString(e));
    return check_tracks(ctx, all, ns_all);
  }
  sf_state* const* states = reg.data();
  const size_t ns = reg.size();
  BatchScratch bs[2];
  sf_status rc = scratch_reserve(ctx, &bs[0], ns, maxseg);
  int active = 1;
  // overlap pays only when a round's tracks can run beside the previous
  // round's other kernels: when some circuit has a range that ends without
  // a measurement (a cut every SF_RANGE_MAX gates); rounds that end in
  // measurements wait for the coin anyway
  bool overlap = false;
  for (size_t i = 0; i < ns && !overlap; ++i) overlap = !states[i]->c->cuts.empty();
  if (ctx->side && overlap) {
    // overlapped rounds: both buffer sets exist before the first launch, and
    // the side stream starts after the work already queued on the context's
    for (size_t i = 0; i < ns && rc == SF_OK; ++i) rc = ensure_second_set(states[i]);
    if (rc == SF_OK) rc = scratch_reserve(ctx, &bs[1], ns, maxseg);
    if (rc == SF_OK && hipEventRecord(ctx->ev_join, ctx->stream) == hipSuccess &&
        hipStreamWaitEvent(ctx->side, ctx->ev_join, 0) == hipSuccess) {
      bool prev_meas = false;
      for (int r = 0; rc == SF_OK && active; ++r) rc = batch_round_ov(ctx, states, ns, bs, &active, r, &prev_meas);
    } else if (rc == SF_OK) {
      rc = fail(ctx, SF_E_DEVICE, "batch run: stream join failed");
    }
    // whatever was queued on the side stream finishes before the context's
    if (hipEventRecord(ctx->ev_join, ctx->side) == hipSuccess)
      (void)hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0);
    (void)hipStreamSynchronize(ctx->side);
  } else {
    while (rc == SF_OK && active) rc = batch_round(ctx, states, ns, &bs[0], &active, 0, true);
  }
  hipError_t e = hipStreamSynchronize(ctx->stream);
  pin_release(ctx);
  scratch_free(ctx, &bs[0]);
  scratch_free(ctx, &bs[1]);
  dfree(ctx, &wj);
  if (rc != SF_OK) return rc;
  if (e != hipSuccess) return fail(ctx, SF_E_DEVICE, "batch run: %s", hipGetErrorString(e));
  return check_tracks(ctx, all, ns_all);
}

extern "C" sf_status sf_batch_run_noalloc(sf_ctx* ctx, sf_state* const* states, size_t ns) {
  if (!ctx || (ns && !states)) return SF_E_INVALID;
  if (any_wide(states, ns)) return fail(ctx, SF_E_INVALID, "frames of more than %d qubits run through sf_run, sf_step "
                                        "and sf_batch_run", SF_NMAX);
  int maxseg = 1;
  for (size_t i = 0; i < ns; ++i) {
    if (!states[i] || states[i]->ctx != ctx) return fail(ctx, SF_E_INVALID, "state %zu is not of this context", i);
    maxseg = std::max(maxseg, states[i]->c->max_segs);
  }
  if (ns == 0) return SF_OK;
  void* base = (ctx->device >= 0 && ctx->device < SF_MAX_DEVICES) ? g_scratch_dev[ctx->device] : nullptr;
  if (!base) return fail(ctx, SF_E_DEVICE, "scratch array of device %d has no address", ctx->device);
  // the largest round: every state active with maxseg segments and a measurement
  const size_t need_d = desc_capacity(ns, maxseg);
  const size_t off_d = desc_offset(ns * sizeof(TrackJob));
  const size_t off_g = desc_offset(off_d + need_d);
  if (off_g + gather_bytes(ns) > SF_SCRATCH_BYTES)
    return fail(ctx, SF_E_TOO_LARGE, "%zu states with up to %d segments need %zu scratch bytes, %zu available", ns,
                maxseg, off_g + gather_bytes(ns), (size_t)SF_SCRATCH_BYTES);
  BatchScratch bs;  // views into the scratch array, never freed
  bs.djobs.p = base;
  bs.djobs.bytes = off_d;
  bs.ddesc.p = (char*)base + off_d;
  bs.ddesc.bytes = need_d;
  sf_status rc = SF_OK;
  int active = 1;
  while (rc == SF_OK && active) rc = batch_round(ctx, states, ns, &bs, &active, 0, false, nullptr, true);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  bs.keep_jobs.clear();
  bs.keep_desc.clear();
  bs.djobs.p = bs.ddesc.p = nullptr;
  if (rc != SF_OK) return rc;
  if (e != hipSuccess) return fail(ctx, SF_E_DEVICE, "batch run: %s", hipGetErrorString(e));
  return check_tracks(ctx, states, ns, (char*)base + off_g);
}

// Re-initialise many states with one kernel launch (their basis states and
// seeds given per state).  Synchronises.
extern "C" sf_status sf_batch_reset(sf_ctx* ctx, sf_state* const* states, size_t ns, const uint64_t* bases,
                                    const uint64_t* seeds) {
  if (!ctx || (ns && !states)) return SF_E_INVALID;
  if (ns == 0) return SF_OK;
  if (any_wide(states, ns)) return fail(ctx, SF_E_INVALID, "frames of more than %d qubits are reset by sf_state_reset",
                                        SF_NMAX);
  for (size_t i = 0; i < ns; ++i)
    if (!states[i] || states[i]->ctx != ctx) return fail(ctx, SF_E_INVALID, "state %zu is not of this context", i);
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t off_p = al(ns * sizeof(InitDesc)), total = off_p + ns * 8 * sizeof(uint64_t);
  DevBuf buf;
  sf_status rc = dalloc(ctx, &buf, total);
  if (rc) return rc;
  std::vector<char> host(total, 0);
  uint64_t* par = (uint64_t*)(host.data() + off_p);
  for (size_t i = 0; i < ns; ++i) {
    sf_state* s = states[i];
    const int W = words_of(s->c->n);
    for (int w = 0; w < W; ++w) par[8 * i + w] = bases ? bases[4 * i + w] : 0;
    par[8 * i + 4] = seeds ? seeds[i] : 0;
    InitDesc d;
    memset(&d, 0, sizeof d);
    d.st = (TrackState*)s->st.p;
    d.amp = (double2*)s->amp[0].p;
    d.flags = (int*)s->flags.p;
    d.params = (const uint64_t*)((char*)buf.p + off_p) + 8 * i;
    d.n = (int)s->c->n;
    memcpy(host.data() + i * sizeof(InitDesc), &d, sizeof d);
  }
  hipError_t e = hipMemcpyAsync(buf.p, host.data(), total, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    prof_begin(ctx, PK_INIT);
    hipLaunchKernelGGL(sf_init_batch, dim3((unsigned)ns), dim3(EB), 0, ctx->stream, (const InitDesc*)buf.p);
    prof_end(ctx);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dfree(ctx, &buf);
  if (e != hipSuccess) return fail(ctx, SF_E_DEVICE, "batch reset: %s", hipGetErrorString(e));
  for (size_t i = 0; i < ns; ++i) {
    set_progress(states[i], Progress{0, 0, 0, 0});
    states[i]->seed = seeds ? seeds[i] : 0;
  }
  return SF_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: for each hull dimension d in [d_lo, d_hi], times the segment
// kernel over 2^d slots at every candidate launch shape (threads per block x
// slots per thread) and keeps the fastest for the elementwise frame kernels.
// The kernels are elementwise, so every shape gives bit-identical results;
// the measurement reductions keep their fixed shape.
// ---------------------------------------------------------------------------
extern "C" sf_status sf_autotune(sf_ctx* ctx, int d_lo, int d_hi, int* blocks, int* grids, float* ms) {
  if (!ctx || d_lo < 0 || d_hi > SF_DMAX - 1 || d_lo > d_hi) return SF_E_INVALID;
  DevBuf amp, sp, had;
  sf_status rc;
  if ((rc = dalloc(ctx, &amp, (size_t)16 << d_hi))) return rc;
  if ((rc = dalloc(ctx, &sp, sizeof(SegProg))) || (rc = dalloc(ctx, &had, sizeof(GF2Q)))) {
    dfree(ctx, &amp);
    dfree(ctx, &sp);
    return rc;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(sf_fill_unit, dim3(grid_for(d_hi)), dim3(EB), 0, ctx->stream, (double2*)amp.p,
                       (uint64_t)1 << d_hi);
    e = hipGetLastError();
  }
  static const int cand_block[] = {64, 128, 256};
  static const int cand_items[] = {1, 2, 4, 8, 16, 32};
  for (int d = d_lo; d <= d_hi && e == hipSuccess; ++d) {
    // a phase-only segment program whose form touches every coordinate
    SegProg h;
    memset(&h, 0, sizeof h);
    h.kind = SEG_NONE;
    h.d = h.d_out = d;
    h.j0 = h.m_j0 = h.meas_index = -1;
    h.ph_re = 1.0;
    h.E.L1 = d ? (uint32_t)((1ull << d) - 1) & 0x55555555u : 0u;
    h.E.L2 = d ? (uint32_t)((1ull << d) - 1) & 0x33333333u : 0u;
    e = hipMemcpyAsync(sp.p, &h, sizeof h, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    const uint64_t N = 1ull << d;
    float best = 1e30f;
    int bb = EB, bg = grid_for(d);
    for (int b : cand_block)
      for (int it : cand_items) {
        if (e != hipSuccess) break;
        uint64_t gq = (N + (uint64_t)b * it - 1) / ((uint64_t)b * it);
        const int g = (int)std::max<uint64_t>(1, std::min<uint64_t>(gq, 65535));
        const int reps = 5;
        hipLaunchKernelGGL(sf_seg_kernel, dim3(g), dim3(b), 0, ctx->stream, (const SegProg*)sp.p,
                           (const GF2Q*)had.p, (double2*)amp.p);
        e = hipEventRecord(e0, ctx->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
          hipLaunchKernelGGL(sf_seg_kernel, dim3(g), dim3(b), 0, ctx->stream, (const SegProg*)sp.p,
                             (const GF2Q*)had.p, (double2*)amp.p);
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        t /= reps;
        if (e == hipSuccess && t < best) { best = t; bb = b; bg = g; }
      }
    if (e != hipSuccess) break;
    ctx->tune_block[d] = bb;
    ctx->tune_grid[d] = bg;
    if (blocks) blocks[d - d_lo] = bb;
    if (grids) grids[d - d_lo] = bg;
    if (ms) ms[d - d_lo] = best;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  dfree(ctx, &amp);
  dfree(ctx, &sp);
  dfree(ctx, &had);
  if (e != hipSuccess) return fail(ctx, SF_E_DEVICE, "autotune: %s", hipGetErrorString(e));
  return SF_OK;
}

static_assert(SF_TUNE_DIMS == SF_DMAX + 1, "tuning table size");

extern "C" sf_status sf_tuning_get(const sf_ctx* ctx, int* blocks, int* grids, int* phase_waves) {
  if (!ctx) return SF_E_INVALID;
  for (int d = 0; d <= SF_DMAX; ++d) {
    if (blocks) blocks[d] = ctx->tune_block[d];
    if (grids) grids[d] = ctx->tune_grid[d];
  }
  if (phase_waves) *phase_waves = ctx->phase_waves;
  return SF_OK;
}

extern "C" sf_status sf_tuning_set(sf_ctx* ctx, const int* blocks, const int* grids, int phase_waves) {
  if (!ctx) return SF_E_INVALID;
  if (phase_waves < 1) return fail(ctx, SF_E_INVALID, "phase wavefront target %d < 1", phase_waves);
  if ((blocks == nullptr) != (grids == nullptr)) return fail(ctx, SF_E_INVALID, "blocks and grids go together");
  if (blocks) {
    for (int d = 0; d <= SF_DMAX; ++d) {
      const int b = blocks[d], g = grids[d];
      if ((b != 64 && b != 128 && b != 256) || g < 1 || g > (1 << 24))
        return fail(ctx, SF_E_INVALID, "shape (%d threads, %d blocks) for d = %d", b, g, d);
    }
    for (int d = 0; d <= SF_DMAX; ++d) {
      ctx->tune_block[d] = blocks[d];
      ctx->tune_grid[d] = grids[d];
    }
  }
  ctx->phase_waves = phase_waves;
  return SF_OK;
}

// ---------------------------------------------------------------------------
// Graph form of a batched run: the launches of a whole run of a fixed set of
// frames (initialisation included) recorded once as a hipGraph of kernel
// nodes and replayed with one launch.  The rounds depend on the circuits
// only, so their descriptors are planned and uploaded when the graph is
// built; basis states and seeds sit in a device table that each replay reads.
// ---------------------------------------------------------------------------
struct sf_graph {
  sf_ctx* ctx;
  std::vector<sf_state*> states;
  std::vector<Progress> final_pr;
  std::vector<uint64_t> params;  // 8 words per frame: basis[4], seed, unused
  DevBuf dparams, ddesc;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// A kernel node after the given nodes (null entries and repeats skipped).
static hipError_t add_node_after(hipGraph_t g, hipGraphNode_t* node, std::initializer_list<hipGraphNode_t> after,
                                 const void* func, dim3 grid, dim3 block, void** args, size_t shmem = 0) {
  hipGraphNode_t deps[4];
  size_t nd = 0;
  for (hipGraphNode_t a : after) {
    if (!a) continue;
    bool seen = false;
    for (size_t t = 0; t < nd; ++t) seen |= deps[t] == a;
    if (!seen && nd < 4) deps[nd++] = a;
  }
  hipKernelNodeParams p;
  memset(&p, 0, sizeof p);
  p.func = const_cast<void*>(func);
  p.gridDim = grid;
  p.blockDim = block;
  p.sharedMemBytes = (unsigned)shmem;
  p.kernelParams = args;
  p.extra = nullptr;
  return hipGraphAddKernelNode(node, g, nd ? deps : nullptr, nd, &p);
}

static void graph_free(sf_graph* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  dfree(g->ctx, &g->dparams);
  dfree(g->ctx, &g->ddesc);
  for (sf_state* s : g->states) s->graph_refs--;
}

extern "C" sf_status sf_batch_graph(sf_ctx* ctx, sf_state* const* states, size_t ns, const uint64_t* const* basis,
                                    const uint64_t* seeds, sf_graph** out) {
  if (!ctx || !out || (ns && !states)) return SF_E_INVALID;
  *out = nullptr;
  for (size_t i = 0; i < ns; ++i)
    if (!states[i] || states[i]->ctx != ctx) return fail(ctx, SF_E_INVALID, "state %zu is not of this context", i);
  if (any_wide(states, ns)) return fail(ctx, SF_E_INVALID, "frames of more than %d qubits run through sf_run, sf_step "
                                        "and sf_batch_run", SF_NMAX);
  {
    std::vector<sf_state*> srt(states, states + ns);
    std::sort(srt.begin(), srt.end());
    if (std::adjacent_find(srt.begin(), srt.end()) != srt.end())
      return fail(ctx, SF_E_INVALID, "a state appears twice in the batch");
  }
  sf_graph* g = new (std::nothrow) sf_graph();
  if (!g) return fail(ctx, SF_E_OOM, "host allocation failed");
  g->ctx = ctx;
  g->states.assign(states, states + ns);
  for (sf_state* s : g->states) s->graph_refs++;
  g->params.assign(8 * std::max<size_t>(1, ns), 0);
  for (size_t i = 0; i < ns; ++i) {
    const int W = (int)((states[i]->c->n + 63) / 64);
    if (basis && basis[i])
      for (int w = 0; w < W; ++w) g->params[8 * i + w] = basis[i][w];
    g->params[8 * i + 4] = seeds ? seeds[i] : 0;
  }
  sf_status rc = dalloc(ctx, &g->dparams, g->params.size() * 8);
  if (rc) { graph_free(g); delete g; return rc; }
  // plan every round from the initial state
  std::vector<Progress> pr(ns, Progress{0, 0, 0, 0});
  std::vector<const uint64_t*> seedp(ns);
  for (size_t i = 0; i < ns; ++i) seedp[i] = (const uint64_t*)g->dparams.p + 8 * i + 4;
  // rounds alternate between the two per-range buffer sets, so that the
  // tracks of a round need not wait for the previous round's element kernels
  for (size_t i = 0; i < ns; ++i)
    if ((rc = ensure_second_set(states[i]))) { graph_free(g); delete g; return rc; }
  std::vector<RoundPlan> rounds;
  for (;;) {
    RoundPlan rp;
    sf_status err;
    if (!plan_round(states, ns, pr.data(), 0, seedp.data(), &rp, &err, nullptr, false, (int)(rounds.size() & 1))) {
      if (err != SF_OK) { graph_free(g); delete g; return err; }
      break;
    }
    rounds.push_back(std::move(rp));
  }
  g->final_pr = pr;
  // one descriptor table: init descriptors, then each round's jobs and descs
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t off_init = 0, total = al(std::max<size_t>(1, ns) * sizeof(InitDesc));
  std::vector<size_t> off_j(rounds.size()), off_d(rounds.size());
  for (size_t r = 0; r < rounds.size(); ++r) {
    off_j[r] = total;
    total += al(rounds[r].jobs.size() * sizeof(TrackJob));
    off_d[r] = total;
    total += al(rounds[r].dbytes.size());
  }
  if ((rc = dalloc(ctx, &g->ddesc, total))) { graph_free(g); delete g; return rc; }
  std::vector<char> host(total, 0);
  for (size_t i = 0; i < ns; ++i) {
    InitDesc d;
    memset(&d, 0, sizeof d);
    d.st = (TrackState*)states[i]->st.p;
    d.amp = (double2*)states[i]->amp[0].p;
    d.flags = (int*)states[i]->flags.p;
    d.params = (const uint64_t*)g->dparams.p + 8 * i;
    d.n = (int)states[i]->c->n;
    memcpy(host.data() + off_init + i * sizeof(InitDesc), &d, sizeof d);
  }
  for (size_t r = 0; r < rounds.size(); ++r) {
    memcpy(host.data() + off_j[r], rounds[r].jobs.data(), rounds[r].jobs.size() * sizeof(TrackJob));
    memcpy(host.data() + off_d[r], rounds[r].dbytes.data(), rounds[r].dbytes.size());
  }
  hipError_t e = hipMemcpyAsync(g->ddesc.p, host.data(), total, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = hipGraphCreate(&g->graph, 0);
  // dependencies as in the overlapped sf_batch_run: the tracks of round r
  // follow the tracks of round r - 1, the element work of round r - 2 (the
  // last user of their buffer set) and the measurement of round r - 1 (its
  // outcomes); the phase, fit, segment and measurement kernels of round r
  // follow the tracks of round r and the element work of round r - 1
  char* base = (char*)g->ddesc.p;
  hipGraphNode_t init = nullptr, track_last = nullptr, elem_last = nullptr, meas_prev = nullptr;
  std::vector<hipGraphNode_t> elem_end(rounds.size(), nullptr);
  if (e == hipSuccess && ns) {
    const InitDesc* di = (const InitDesc*)(base + off_init);
    void* args[] = {(void*)&di};
    e = add_node_after(g->graph, &init, {}, (const void*)sf_init_batch, dim3((unsigned)ns), dim3(EB), args);
    track_last = elem_last = init;
  }
  for (size_t r = 0; r < rounds.size() && e == hipSuccess; ++r) {
    const RoundPlan& rp = rounds[r];
    const int na = rp.na;
    const TrackJob* dj = (const TrackJob*)(base + off_j[r]);
    const ElemDesc* dd = (const ElemDesc*)(base + off_d[r]);
    const hipGraphNode_t reuse = r >= 2 ? elem_end[r - 2] : nullptr;
    int off = 0;
    for (int w = 1; w <= SF_WMAX && e == hipSuccess; ++w) {
      if (!rp.wcount[w]) continue;
      const TrackJob* djw = dj + off;
      void* args[] = {(void*)&djw};
      hipGraphNode_t nd = nullptr;
      e = add_node_after(g->graph, &nd, {track_last, reuse, meas_prev}, track_many_fn(w), dim3(rp.wcount[w]),
                         dim3(TL), args);
      if (e == hipSuccess) track_last = nd;
      off += rp.wcount[w];
    }
    // element chain of this round
    hipGraphNode_t prev = elem_last;
    bool first = true;
    auto chain = [&](const void* func, dim3 grid, dim3 block, void** args, size_t shmem = 0) {
      hipGraphNode_t nd = nullptr;
      if (first)
        e = add_node_after(g->graph, &nd, {prev, track_last}, func, grid, block, args, shmem);
      else
        e = add_node_after(g->graph, &nd, {prev}, func, grid, block, args, shmem);
      if (e == hipSuccess) { prev = nd; first = false; }
    };
    off = 0;
    for (int w = 1; w <= SF_WMAX && e == hipSuccess; ++w) {
      if (!rp.wcount[w]) continue;
      const TrackJob* djw = dj + off;
      void* args[] = {(void*)&djw};
      if (rp.wchunk[w] > 0) {
        chain(phase_many_fn(w), dim3(rp.wchunk[w], rp.wcount[w]), dim3(TL), args,
              rp.anym ? 0 : SF_PHASE_PAD_BESIDE);
        if (e == hipSuccess && rp.wseg[w] > 0)
          chain((const void*)sf_fit_many, dim3(rp.wseg[w], rp.wcount[w]), dim3(TL), args);
      }
      off += rp.wcount[w];
    }
    if (rp.msmall) {
      if ((rp.kmax > 0 || rp.anym) && e == hipSuccess) {
        const ElemDesc* d0 = dd;
        int kmax = rp.kmax, nna = na, meas = rp.anym ? 1 : 0;
        void* args[] = {(void*)&d0, (void*)&kmax, (void*)&nna, (void*)&meas};
        chain((const void*)sf_elem_small_batch, dim3(na), dim3(EB), args);
      }
    } else {
      int nna = na;
      for (int k = 0; k < rp.kmax && e == hipSuccess; ++k) {
        if (!row_blocks(rp, k)) continue;
        const ElemDesc* dk = dd;
        const uint32_t* bk = row_starts(rp, dd, k);
        int kk = k;
        void* args[] = {(void*)&dk, (void*)&bk, (void*)&nna, (void*)&kk};
        chain((const void*)sf_seg_batch, dim3(row_blocks(rp, k)), dim3(EB), args);
      }
      if (rp.anym && e == hipSuccess) {
        const ElemDesc* dm = dd;
        const uint32_t* rb = row_starts(rp, dd, rp.kmax);
        const uint32_t* fb = row_starts(rp, dd, rp.kmax + 1);
        void* rargs[] = {(void*)&dm, (void*)&rb, (void*)&nna};
        void* cargs[] = {(void*)&dm};
        void* fargs[] = {(void*)&dm, (void*)&fb, (void*)&nna};
        const dim3 fg(row_blocks(rp, rp.kmax + 1));
        chain((const void*)sf_meas_reduce_batch, dim3(row_blocks(rp, rp.kmax)), dim3(EB), rargs);
        if (e == hipSuccess && coin_apart(rp)) {
          chain((const void*)sf_meas_coin_batch, dim3(na), dim3(EB), cargs);
          if (e == hipSuccess) chain((const void*)sf_meas_apply_batch, fg, dim3(EB), fargs);
        } else if (e == hipSuccess) {
          chain((const void*)sf_meas_filter_batch, fg, dim3(EB), fargs);
        }
      }
    }
    if (first && e == hipSuccess) {
      // no element work this round: the round ends with its tracks
      prev = track_last;
    }
    elem_last = prev;
    elem_end[r] = prev;
    meas_prev = rp.anym ? prev : nullptr;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    graph_free(g);
    delete g;
    return fail(ctx, SF_E_DEVICE, "graph build: %s", hipGetErrorString(e));
  }
  *out = g;
  return SF_OK;
}

extern "C" sf_status sf_graph_set_input(sf_graph* g, size_t i, const uint64_t* basis, uint64_t seed) {
  if (!g) return SF_E_INVALID;
  if (i >= g->states.size()) return fail(g->ctx, SF_E_INVALID, "frame %zu of %zu", i, g->states.size());
  const int W = (int)((g->states[i]->c->n + 63) / 64);
  for (int w = 0; w < 4; ++w) g->params[8 * i + w] = (basis && w < W) ? basis[w] : 0;
  g->params[8 * i + 4] = seed;
  return SF_OK;
}

extern "C" sf_status sf_graph_launch(sf_graph* g) {
  if (!g) return SF_E_INVALID;
  sf_ctx* ctx = g->ctx;
  HIPCHK(ctx, hipMemcpyAsync(g->dparams.p, g->params.data(), g->params.size() * 8, hipMemcpyHostToDevice,
                             ctx->stream));
  HIPCHK(ctx, hipGraphLaunch(g->exec, ctx->stream));
  for (size_t i = 0; i < g->states.size(); ++i) {
    set_progress(g->states[i], g->final_pr[i]);
    g->states[i]->seed = g->params[8 * i + 4];
  }
  return SF_OK;
}

extern "C" sf_status sf_graph_destroy(sf_graph* g) {
  if (!g) return SF_OK;
  (void)hipStreamSynchronize(g->ctx->stream);
  graph_free(g);
  delete g;
  return SF_OK;
}

// ---------------------------------------------------------------------------
// Serving: a request loop with continuous batching.  Jobs are admitted in
// arrival order while their projected device bytes fit the budget and a slot
// is free; every tick runs one batched round (each resident frame advances to
// its next measurement or to its end), then finished jobs are reported.  A job
// that arrives while others run joins at the next tick.
// ---------------------------------------------------------------------------
struct ServeJob {
  uint64_t id;
  const sf_circuit* c;
  std::vector<uint64_t> basis;
  uint64_t seed;
  sf_state* st;
  int status;       // 0 queued, 1 resident, 2 done, 3 cancelled, 4 failed
  uint32_t passed;  // ticks in which a later job was admitted ahead of it
};

// A queued job that does not fit yet may be passed by later jobs that do, for
// at most this many ticks; after that nothing behind it is admitted until it
// is (so a large job is not starved by a stream of small ones).
#define SF_SERVE_MAX_PASS 16

struct sf_server {
  sf_ctx* ctx;
  uint64_t budget, used;
  uint32_t max_resident;
  int tick_segments;
  uint64_t next_id;
  std::vector<ServeJob*> queue;     // waiting, arrival order
  std::vector<ServeJob*> resident;  // admitted, running
  std::unordered_map<uint64_t, ServeJob*> jobs;  // every job not yet released
  BatchScratch bs;
  uint64_t ticks, admitted, rejected;
};

extern "C" sf_status sf_serve_create(sf_ctx* ctx, uint64_t budget_bytes, uint32_t max_resident,
                                     uint32_t tick_segments, sf_server** out) {
  if (!ctx || !out || max_resident == 0 || tick_segments > (1u << 30)) return SF_E_INVALID;
  sf_server* sv = new (std::nothrow) sf_server();
  if (!sv) return fail(ctx, SF_E_OOM, "host allocation failed");
  sv->ctx = ctx;
  sv->budget = budget_bytes;
  sv->used = 0;
  sv->max_resident = max_resident;
  sv->tick_segments = (int)tick_segments;
  sv->next_id = 1;
  sv->ticks = sv->admitted = sv->rejected = 0;
  *out = sv;
  return SF_OK;
}

static ServeJob* find_job(sf_server* sv, uint64_t id) {
  auto it = sv->jobs.find(id);
  return it == sv->jobs.end() ? nullptr : it->second;
}

extern "C" sf_status sf_serve_submit(sf_server* sv, const sf_circuit* c, const uint64_t* basis, uint64_t seed,
                                     uint64_t* job_id) {
  if (!sv || !c || !job_id) return SF_E_INVALID;
  if (c->wide) return fail(sv->ctx, SF_E_INVALID, "frames of more than %d qubits run through sf_run, sf_step and "
                           "sf_batch_run", SF_NMAX);
  if (sv->budget && c->projected > sv->budget) {
    sv->rejected++;
    return fail(sv->ctx, SF_E_TOO_LARGE, "job needs %llu bytes, budget is %llu",
                (unsigned long long)c->projected, (unsigned long long)sv->budget);
  }
  ServeJob* j = new (std::nothrow) ServeJob();
  if (!j) return fail(sv->ctx, SF_E_OOM, "host allocation failed");
  j->id = sv->next_id++;
  j->c = c;
  const int W = (int)((c->n + 63) / 64);
  j->basis.assign(W, 0);
  if (basis)
    for (int w = 0; w < W; ++w) j->basis[w] = basis[w];
  j->seed = seed;
  j->st = nullptr;
  j->status = 0;
  j->passed = 0;
  sv->queue.push_back(j);
  sv->jobs[j->id] = j;
  *job_id = j->id;
  return SF_OK;
}

// Admission: queued jobs in arrival order, each admitted when its projected
// bytes fit the budget and a resident slot is free.  A job that does not fit
// is passed over (later jobs may still be admitted) unless it has been passed
// SF_SERVE_MAX_PASS times.  A job whose state cannot be allocated waits while
// others are resident (they will free memory) and fails when none is.
static void serve_admit(sf_server* sv) {
  sf_ctx* ctx = sv->ctx;
  std::vector<ServeJob*> waiting;
  bool blocked = false;  // an old job is waiting: admit nothing behind it
  bool passed = false;   // a job was admitted ahead of the oldest waiting one
  ServeJob* first_passed = nullptr;
  for (size_t qi = 0; qi < sv->queue.size(); ++qi) {
    ServeJob* j = sv->queue[qi];
    bool fits = !blocked && sv->resident.size() < sv->max_resident &&
                !(sv->budget && sv->used + j->c->projected > sv->budget);
    if (fits) {
      sf_status rc = sf_state_init(ctx, j->c, j->basis.data(), j->seed, &j->st);
      if ((rc == SF_E_OOM || rc == SF_E_TOO_LARGE) && !sv->resident.empty()) {
        fits = false;
      } else if (rc != SF_OK) {
        j->st = nullptr;
        j->status = 4;
        continue;
      }
    }
    if (!fits) {
      waiting.push_back(j);
      if (!first_passed) first_passed = j;
      if (j->passed >= SF_SERVE_MAX_PASS) blocked = true;
      continue;
    }
    j->status = 1;
    sv->used += j->c->projected;
    sv->admitted++;
    sv->resident.push_back(j);
    passed |= first_passed != nullptr;
  }
  if (passed) first_passed->passed++;
  sv->queue.swap(waiting);
}

// A resident job whose round could not be planned (its buffers could not be
// allocated, or it ran out of room): it fails, keeps its budget share until
// released, and the others go on.
static void serve_fail_resident(sf_server* sv, size_t idx) {
  ServeJob* j = sv->resident[idx];
  j->status = 4;
  sv->resident.erase(sv->resident.begin() + (long)idx);
}

extern "C" sf_status sf_serve_tick(sf_server* sv, uint32_t* n_resident, uint32_t* n_queued) {
  if (!sv) return SF_E_INVALID;
  sf_ctx* ctx = sv->ctx;
  serve_admit(sv);
  while (!sv->resident.empty()) {
    std::vector<sf_state*> sts;
    int maxseg = 1;
    for (ServeJob* j : sv->resident) { sts.push_back(j->st); maxseg = std::max(maxseg, j->c->max_segs); }
    sf_status rc = scratch_reserve(ctx, &sv->bs, sts.size(), maxseg);
    if (rc != SF_OK) return rc;
    int active = 0, bad = -1;
    rc = batch_round(ctx, sts.data(), sts.size(), &sv->bs, &active, sv->tick_segments, false, &bad);
    if (rc != SF_OK && bad >= 0) {
      // nothing was queued: drop the offending job and plan again
      serve_fail_resident(sv, (size_t)bad);
      continue;
    }
    hipError_t e = hipStreamSynchronize(ctx->stream);
    sv->bs.keep_jobs.clear();
    sv->bs.keep_desc.clear();
    if (rc != SF_OK) return rc;
    if (e != hipSuccess) return fail(ctx, SF_E_DEVICE, "serve tick: %s", hipGetErrorString(e));
    std::vector<ServeJob*> still;
    for (ServeJob* j : sv->resident) {
      if (j->st->orig_done >= j->c->orig_end.size()) {
        j->status = check_track(j->st) == SF_OK ? 2 : 4;
      } else {
        still.push_back(j);
      }
    }
    sv->resident.swap(still);
    break;
  }
  sv->ticks++;
  if (n_resident) *n_resident = (uint32_t)sv->resident.size();
  if (n_queued) *n_queued = (uint32_t)sv->queue.size();
  return SF_OK;
}

extern "C" sf_status sf_serve_poll(sf_server* sv, uint64_t job_id, int* status, sf_state** state) {
  if (!sv || !status) return SF_E_INVALID;
  ServeJob* j = find_job(sv, job_id);
  if (!j) return fail(sv->ctx, SF_E_INVALID, "unknown job %llu", (unsigned long long)job_id);
  *status = j->status;
  if (state) *state = j->status == 2 ? j->st : nullptr;
  return SF_OK;
}

// Free a finished, failed or queued job's state and its budget share.
extern "C" sf_status sf_serve_release(sf_server* sv, uint64_t job_id) {
  if (!sv) return SF_E_INVALID;
  ServeJob* j = find_job(sv, job_id);
  if (!j) return fail(sv->ctx, SF_E_INVALID, "unknown job %llu", (unsigned long long)job_id);
  if (j->status == 1) return fail(sv->ctx, SF_E_STATE, "job %llu is running", (unsigned long long)job_id);
  if (j->st) {
    sf_state_destroy(j->st);
    j->st = nullptr;
    if (j->status == 2 || j->status == 4) sv->used -= j->c->projected;
  }
  for (size_t i = 0; i < sv->queue.size(); ++i)
    if (sv->queue[i] == j) { sv->queue.erase(sv->queue.begin() + i); break; }
  sv->jobs.erase(j->id);
  delete j;
  return SF_OK;
}

// Cancel a queued or resident job; its slot and budget share free at once.
extern "C" sf_status sf_serve_cancel(sf_server* sv, uint64_t job_id) {
  if (!sv) return SF_E_INVALID;
  ServeJob* j = find_job(sv, job_id);
  if (!j) return fail(sv->ctx, SF_E_INVALID, "unknown job %llu", (unsigned long long)job_id);
  if (j->status == 0) {
    for (size_t i = 0; i < sv->queue.size(); ++i)
      if (sv->queue[i] == j) { sv->queue.erase(sv->queue.begin() + i); break; }
  } else if (j->status == 1) {
    for (size_t i = 0; i < sv->resident.size(); ++i)
      if (sv->resident[i] == j) { sv->resident.erase(sv->resident.begin() + i); break; }
    sf_state_destroy(j->st);
    j->st = nullptr;
    sv->used -= j->c->projected;
  } else {
    return SF_OK;
  }
  j->status = 3;
  return SF_OK;
}

extern "C" sf_status sf_serve_stats(sf_server* sv, uint64_t* ticks, uint64_t* admitted, uint64_t* rejected,
                                    uint64_t* used_bytes) {
  if (!sv) return SF_E_INVALID;
  if (ticks) *ticks = sv->ticks;
  if (admitted) *admitted = sv->admitted;
  if (rejected) *rejected = sv->rejected;
  if (used_bytes) *used_bytes = sv->used;
  return SF_OK;
}

extern "C" sf_status sf_serve_destroy(sf_server* sv) {
  if (!sv) return SF_OK;
  for (auto& kv : sv->jobs) {
    if (kv.second->st) sf_state_destroy(kv.second->st);
    delete kv.second;
  }
  scratch_free(sv->ctx, &sv->bs);
  delete sv;
  return SF_OK;
}
