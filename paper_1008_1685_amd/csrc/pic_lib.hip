// Host side of the C ABI declared in include/pic.h (and, through
// pic2d_host.inc at the end, include/pic2d.h): workspace carving,
// validation, kernel launches, state I/O and per-kernel event timing.
#include "pic.h"
#include "kernels.hpp"

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace pic;

// Histogram counters of pic_spectrum_static: a fixed device array, so that
// entry point needs no device memory from the caller or the allocator.  Each
// device that calls it holds its own copy until the process ends.  In host
// code this name is not a device address: host code uses the per-device
// address from hipGetSymbolAddress (static_scratch below).
constexpr int kStaticSpectrumBins = 1 << 16;  // 512 KiB of 64-bit counters
static __device__ __align__(256) unsigned long long scratch[kStaticSpectrumBins];

namespace {

thread_local std::string g_err;

pic_status fail(pic_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(PIC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

constexpr double kRe_um = 2.8179403262e-9;  // classical electron radius (um)
constexpr double kMec2_MeV = 0.51099895;
constexpr int kMaxSpectrumBins = 1 << 16;

// Bump allocator over the caller's workspace (or a size counter when base is null).
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

struct Derived {
  int nx, c0, nf;
  double dx, dt, eps, w_ref;
  long long n_foil, cap;
  int prec;
  size_t rsize;
};

pic_status derive(const pic_config* c, Derived* d) {
  if (!c) return fail(PIC_EINVAL, "null config");
  if (c->struct_size != sizeof(pic_config))
    return fail(PIC_EINVAL, "pic_config.struct_size mismatch (ABI version)");
  if (c->precision != PIC_FP32 && c->precision != PIC_FP64)
    return fail(PIC_EINVAL, "precision must be PIC_FP32 or PIC_FP64");
  if (!(c->lambda_um > 0)) return fail(PIC_EINVAL, "lambda_um must be > 0");
  if (c->cells_per_lambda < 4) return fail(PIC_EINVAL, "cells_per_lambda must be >= 4");
  if (c->ppc < 1) return fail(PIC_EINVAL, "ppc must be >= 1");
  if (!(c->cfl > 0 && c->cfl <= 0.5)) return fail(PIC_EINVAL, "cfl must be in (0, 0.5]");
  if (c->pol != PIC_LP && c->pol != PIC_CP) return fail(PIC_EINVAL, "pol must be PIC_LP or PIC_CP");
  if (!(c->t_rise >= 0 && c->t_flat >= 0 && c->t_fall >= 0))
    return fail(PIC_EINVAL, "envelope times must be >= 0");
  if (!(c->n0 >= 0) || !(c->mass_ratio > 0) || !(c->jitter >= 0 && c->jitter <= 1))
    return fail(PIC_EINVAL, "n0 >= 0, mass_ratio > 0, jitter in [0, 1] required");
  if (!(c->n0 > 0)) return fail(PIC_EINVAL, "n0 must be > 0 (it sets the particle weight)");
  if (c->sort_interval < 1) return fail(PIC_EINVAL, "sort_interval must be >= 1");
  if (!std::isfinite(c->a0)) return fail(PIC_EINVAL, "a0 must be finite");
  const int cpl = c->cells_per_lambda;
  const double nxd = std::llround(c->box_lambda * cpl);
  if (!(nxd >= 8 && nxd <= (1 << 27))) return fail(PIC_EINVAL, "box must hold 8 .. 2^27 cells");
  d->nx = (int)nxd;
  d->c0 = (int)std::llround(c->x_foil * cpl);
  d->nf = (int)std::llround(c->thickness * cpl);
  if (d->c0 < 0 || d->nf < 0 || d->c0 + d->nf > d->nx)
    return fail(PIC_EINVAL, "foil must lie inside the box");
  d->dx = 2.0 * M_PI / cpl;
  d->dt = c->cfl * d->dx;
  d->eps = 4.0 * M_PI / 3.0 * kRe_um / c->lambda_um;
  d->w_ref = c->n0 * d->dx / c->ppc;
  d->n_foil = (long long)d->nf * c->ppc;
  if (c->capacity < 0) return fail(PIC_EINVAL, "capacity must be >= 0 (0: the foil's count)");
  d->cap = std::max<long long>(d->n_foil, c->capacity);
  // kernels address particle arrays with 32-bit byte offsets
  const long long elem = c->precision == PIC_FP32 ? 4 : 8;
  if (d->cap < 0 || d->cap * elem > (1ll << 32) - (long long)std::max(kTile, kBatchTile) * elem)
    return fail(PIC_EINVAL, "capacity per species too large (arrays must stay below 4 GiB)");
  d->prec = c->precision;
  d->rsize = c->precision == PIC_FP32 ? sizeof(float) : sizeof(double);
  return PIC_OK;
}

struct SpeciesBuf {
  int* cell;
  void* off;
  void* ux;
  void* uy;
  void* uz;
  void* w;
  float* rx;
  float* ry;
  float* rz;
};

struct TimingRec {
  hipEvent_t a, b;
  int kind;
  bool used;
};

}  // namespace

struct pic_run {
  pic_config cfg;
  Derived d;
  long long n_max[2];   // host upper bound of particles per species
  long long step;
  int pp;               // particle buffer (and count slot) parity
  // device memory carved from the workspace
  SpeciesBuf sp[2][2];  // [species][parity]
  void* FN[2];          // [parity] node fields (E_y, E_z)
  void* FH[2];          // [parity] half-node fields (E_x, B_y, B_z, 0)
  unsigned long long* J[2][3];
  long long* Ex_int;
  long long* count;     // [parity][species]
  long long* step_dev;
  int* flags;
  double* acc;          // [tiles][4]
  int* trange;          // [2 parities][tiles][2]: tile cell ranges left by the push
  int* tpred;           // [2 parities]: the ranges of that parity match the particles
  double* budget;       // [4]
  int* cnt[2];
  int* cursor[2];
  long long* rho;
  double* part;
  long long* ipart;
  DiagOutDev* dout;
  unsigned long long* hist;
  int tiles_max;
  int push_tile = kTile;  // particles per push work-group: kTile, or kBatchTile for small runs
  struct pic_batch* batch = nullptr;  // set while the run is stepped by a batch
  // pic_step replays two sort intervals at a time as one captured graph (the
  // kernel arguments repeat with that period: step parity and sort parity
  // both return); one graph per (sort parity, step parity) at its start
  hipGraphExec_t step_graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipGraph_t step_graph_def[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipStream_t capture_stream = nullptr;  // a stream to record on; replays go to the caller's
  // work-groups per launch of the push and sort passes (0: one launch per
  // pass); a large run split this way lets other streams' kernels in between
  int max_grid = 0;
  // timing: every timing-th launch of each kernel kind is bracketed by events
  int timing = 0;
  long long seen[3] = {0, 0, 0};
  std::vector<TimingRec> ev;
  size_t ev_next = 0;
  double ms[3] = {0, 0, 0};
  long long launches[3] = {0, 0, 0};
};

namespace {

int tiles_for(long long n, int tile = kTile) { return (int)((n + tile - 1) / tile); }

void carve(pic_run* r, Carver& cv) {
  const Derived& d = r->d;
  const size_t rs = d.rsize;
  const bool comp = r->cfg.precision == PIC_FP32 && r->cfg.rr && r->cfg.rr_compensated;
  for (int s = 0; s < 2; ++s)
    for (int p = 0; p < 2; ++p) {
      SpeciesBuf& b = r->sp[s][p];
      b.cell = cv.take<int>(d.cap);
      b.off = cv.take<char>(d.cap * rs);
      b.ux = cv.take<char>(d.cap * rs);
      b.uy = cv.take<char>(d.cap * rs);
      b.uz = cv.take<char>(d.cap * rs);
      b.w = cv.take<char>(d.cap * rs);
      b.rx = b.ry = b.rz = nullptr;
      if (s == 0 && comp) {
        b.rx = cv.take<float>(d.cap);
        b.ry = cv.take<float>(d.cap);
        b.rz = cv.take<float>(d.cap);
      }
    }
  for (int p = 0; p < 2; ++p) {
    r->FN[p] = cv.take<char>((size_t)(d.nx + 1) * 2 * rs);
    r->FH[p] = cv.take<char>((size_t)(d.nx + 2) * 4 * rs);
  }
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < 3; ++k) r->J[p][k] = cv.take<unsigned long long>(d.nx + 3);
  r->Ex_int = cv.take<long long>(d.nx + 2);
  r->count = cv.take<long long>(4);
  r->step_dev = cv.take<long long>(1);
  r->flags = cv.take<int>(4);
  r->tiles_max = 2 * tiles_for(d.cap, kMinTile);  // a run may also step in a batch
  r->acc = cv.take<double>(4 * (size_t)std::max(r->tiles_max, 1));
  r->trange = cv.take<int>(4 * (size_t)std::max(r->tiles_max, 1));
  r->tpred = cv.take<int>(2);
  r->budget = cv.take<double>(4);
  for (int s = 0; s < 2; ++s) {
    r->cnt[s] = cv.take<int>(d.nx + 1);
    r->cursor[s] = cv.take<int>(d.nx + 1);
  }
  r->rho = cv.take<long long>(d.nx + 3);
  r->part = cv.take<double>(2 * kDiagPartBlocks + 3 * kDiagFieldBlocks);
  r->ipart = cv.take<long long>(kDiagFieldBlocks + 2 * kDiagPartBlocks);
  r->dout = cv.take<DiagOutDev>(1);
  r->hist = cv.take<unsigned long long>(kMaxSpectrumBins);
}

template <typename R>
SpeciesDev<R> dev(const SpeciesBuf& b) {
  return SpeciesDev<R>{b.cell, (R*)b.off, (R*)b.ux, (R*)b.uy, (R*)b.uz, (R*)b.w, b.rx, b.ry, b.rz};
}

template <typename R>
FieldsDev<R> fdev(const pic_run* r, int parity) {
  return FieldsDev<R>{(NodeF<R>*)r->FN[parity], (HalfF<R>*)r->FH[parity]};
}

__global__ void k_set_counts(long long* dst, long long a, long long b) {
  dst[0] = a;
  dst[1] = b;
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

constexpr size_t kNoEvent = ~(size_t)0;

// Events for a sampled launch: the kernel launch itself records them at its
// start and end (hipExtLaunchKernel), so the measured time is the kernel's
// execution without the queue time of separate event packets.
// The ring of event pairs, created once, when timing is switched on (not at
// the first sampled launch, where creating them would fall inside the timed
// stretch).
template <class Run>
pic_status ev_create(Run* r) {
  if (!r->ev.empty()) return PIC_OK;
  r->ev.resize(512);
  for (auto& e : r->ev) {
    HIP_TRY(hipEventCreate(&e.a));
    HIP_TRY(hipEventCreate(&e.b));
    e.used = false;
  }
  return PIC_OK;
}

template <class Run>
pic_status ev_pick(Run* r, int kind, size_t* slot, hipEvent_t* a, hipEvent_t* b) {
  *slot = kNoEvent;
  *a = *b = nullptr;
  if (!r->timing) return PIC_OK;
  if (r->seen[kind]++ % r->timing) return PIC_OK;  // not sampled
  pic_status ps = ev_create(r);
  if (ps) return ps;
  TimingRec& e = r->ev[r->ev_next];
  if (e.used) {  // ring full: fold the oldest record in
    HIP_TRY(hipEventSynchronize(e.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e.a, e.b));
    r->ms[e.kind] += ms;
    e.used = false;
  }
  e.kind = kind;
  *slot = r->ev_next;
  *a = e.a;
  *b = e.b;
  r->ev_next = (r->ev_next + 1) % r->ev.size();
  return PIC_OK;
}

template <class Run>
void ev_done(Run* r, size_t slot) {
  if (slot == kNoEvent) return;
  TimingRec& e = r->ev[slot];
  e.used = true;
  r->launches[e.kind] += 1;
}

bool comp_on(const pic_run* r) {
  return r->cfg.rr && r->cfg.rr_compensated && r->cfg.precision == PIC_FP32;
}

int sort_blocks_for(long long n) {
  return (int)std::max<long long>(1, (n + kSortTile - 1) / kSortTile);
}

// Kernel arguments of run r for particle buffer parity pp and field parity fp.
template <typename R>
PushArgs<R> make_push_args(const pic_run* r, int pp, int fp, int tile = kTile) {
  const Derived& d = r->d;
  PushArgs<R> a{};
  for (int s = 0; s < 2; ++s) a.sp[s] = dev<R>(r->sp[s][pp]);
  a.count = r->count + 2 * pp;
  a.tiles0 = tiles_for(r->n_max[0], tile);
  a.f = fdev<R>(r, fp);
  for (int k = 0; k < 3; ++k) a.J[k] = r->J[fp][k];
  a.acc = r->acc;
  a.flags = r->flags;
  a.nx = d.nx;
  a.cfl = (R)r->cfg.cfl;
  a.dt = (R)d.dt;
  a.eps = (R)d.eps;
  a.qh[0] = (R)(-1.0 * d.dt * 0.5);
  a.qh[1] = (R)(1.0 / r->cfg.mass_ratio * d.dt * 0.5);
  a.Z[0] = -1;
  a.Z[1] = 1;
  a.mass[0] = 1.0;
  a.mass[1] = r->cfg.mass_ratio;
  a.rr0 = r->cfg.rr != 0;
  a.comp = comp_on(r) ? 1 : 0;
  a.sw = (R)(256.0 / d.w_ref);
  for (int s = 0; s < 2; ++s)  // the kernel's own rounding of a particle of weight w_ref
    a.qw_ref[s] = a.Z[s] * (int)std::rint((R)d.w_ref * a.sw);
  a.ntiles = a.tiles0 + tiles_for(r->n_max[1], tile);
  const size_t rt = 2 * (size_t)std::max(r->tiles_max, 1);
  a.rng_in = r->trange + fp * rt;
  a.rng_out = r->trange + (fp ^ 1) * rt;
  a.pred_in = r->tpred + fp;
  a.pred_out = r->tpred + (fp ^ 1);
  return a;
}

template <typename R>
FieldArgs<R> make_field_args(const pic_run* r, int p, int tick) {
  const Derived& d = r->d;
  FieldArgs<R> f{};
  f.in = fdev<R>(r, p);
  f.out = fdev<R>(r, p ^ 1);
  for (int k = 0; k < 3; ++k) {
    f.J[k] = (const long long*)r->J[p][k];
    f.Jnext[k] = r->J[p ^ 1][k];
  }
  f.Ex_int = r->Ex_int;
  f.budget = r->budget;
  f.step = r->step_dev;
  f.tick = tick;
  f.nx = d.nx;
  f.a = (R)r->cfg.cfl;
  f.dt = (R)d.dt;
  f.dtd = d.dt;
  const double sE = d.w_ref * std::ldexp(1.0, -32);
  f.sEx = sE;
  f.sJx = sE / d.dt;
  f.sJy = sE / d.dx;
  const bool lp = r->cfg.pol == PIC_LP;
  f.ay = lp ? r->cfg.a0 : r->cfg.a0 / std::sqrt(2.0);
  f.az = lp ? 0.0 : r->cfg.a0 / std::sqrt(2.0);
  f.tr = 2.0 * M_PI * r->cfg.t_rise;
  f.tf = 2.0 * M_PI * r->cfg.t_flat;
  f.tl = 2.0 * M_PI * r->cfg.t_fall;
  return f;
}

int field_blocks_for(const pic_run* r) { return (r->d.nx + 3 + kFieldChunk - 1) / kFieldChunk; }

template <typename R>
SortArgs<R> make_sort_args(const pic_run* r, int pp) {
  SortArgs<R> p{};
  for (int s = 0; s < 2; ++s) {
    p.src[s] = dev<R>(r->sp[s][pp]);
    p.dst[s] = dev<R>(r->sp[s][pp ^ 1]);
    p.cnt[s] = r->cnt[s];
    p.cursor[s] = r->cursor[s];
  }
  p.count = r->count + 2 * pp;
  p.nx = r->d.nx;
  p.comp = comp_on(r) ? 1 : 0;
  p.blocks0 = sort_blocks_for(r->n_max[0]);
  p.pred = r->tpred;
  return p;
}

// Launches of one step's kernels.  `capture`: the launch is being recorded
// into a graph (plain launches, no timing events).
// Launches covering `total` work-groups: one, or pieces of at most max_grid.
template <class F>
void split_launch(int total, int max_grid, F&& launch) {
  const int step = max_grid > 0 ? max_grid : total;
  for (int b0 = 0; b0 < total; b0 += step) launch(b0, std::min(step, total - b0), b0 == 0, b0 + step >= total);
}

template <typename R>
pic_status launch_push(pic_run* r, hipStream_t st, bool capture = false) {
  PushArgs<R> a = make_push_args<R>(r, r->pp, (int)(r->step & 1), r->push_tile);
  if (a.ntiles == 0) return PIC_OK;
  size_t slot = kNoEvent;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!capture) {
    pic_status ps = ev_pick(r, 0, &slot, &e0, &e1);
    if (ps) return ps;
  }
  // the events span the pieces: start of the first, end of the last
  split_launch(a.ntiles, r->max_grid, [&](int t0, int n, bool first, bool last) {
    a.tile0 = t0;
    hipEvent_t s0 = first ? e0 : nullptr, s1 = last ? e1 : nullptr;
    const bool small = r->push_tile == kBatchTile;
    if (capture && small)  // (recorded launches carry no events)
      hipLaunchKernelGGL(k_push_small<R>, dim3(n), dim3(kThreads), 0, st, a);
    else if (capture)
      hipLaunchKernelGGL(k_push<R>, dim3(n), dim3(kThreads), 0, st, a);
    else if (small)
      hipExtLaunchKernelGGL(k_push_small<R>, dim3(n), dim3(kThreads), 0, st, s0, s1, 0, a);
    else
      hipExtLaunchKernelGGL(k_push<R>, dim3(n), dim3(kThreads), 0, st, s0, s1, 0, a);
  });
  HIP_TRY(hipGetLastError());
  if (!capture) ev_done(r, slot);
  return PIC_OK;
}

template <typename R>
pic_status launch_field(pic_run* r, hipStream_t st, bool capture = false) {
  const FieldArgs<R> f = make_field_args<R>(r, (int)(r->step & 1), 1);
  if (capture) {
    hipLaunchKernelGGL(k_field<R>, dim3(field_blocks_for(r)), dim3(kFieldChunk), 0, st, f);
  } else {
    size_t slot;
    hipEvent_t e0, e1;
    pic_status ps = ev_pick(r, 1, &slot, &e0, &e1);
    if (ps) return ps;
    hipExtLaunchKernelGGL(k_field<R>, dim3(field_blocks_for(r)), dim3(kFieldChunk), 0, st, e0, e1, 0, f);
    ev_done(r, slot);
  }
  HIP_TRY(hipGetLastError());
  r->step += 1;
  return PIC_OK;
}

template <typename R>
pic_status launch_sort(pic_run* r, hipStream_t st, bool capture = false) {
  const SortArgs<R> p = make_sort_args<R>(r, r->pp);
  const int grid = p.blocks0 + sort_blocks_for(r->n_max[1]);
  size_t slot = kNoEvent;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!capture) {
    pic_status ps = ev_pick(r, 2, &slot, &e0, &e1);
    if (ps) return ps;
  }
  // the events span the three passes: start of the histogram, end of the scatter
  SortArgs<R> q = p;
  split_launch(grid, r->max_grid, [&](int b0, int n, bool first, bool) {
    q.blk0 = b0;
    if (capture)
      hipLaunchKernelGGL(k_sort_hist<R>, dim3(n), dim3(kSortThreads), 0, st, q);
    else
      hipExtLaunchKernelGGL(k_sort_hist<R>, dim3(n), dim3(kSortThreads), 0, st, first ? e0 : nullptr,
                            nullptr, 0, q);
  });
  hipLaunchKernelGGL(k_sort_scan, dim3(2), dim3(1024), 0, st, r->cnt[0], r->cnt[1], r->cursor[0],
                     r->cursor[1], r->count + 2 * (r->pp ^ 1), r->d.nx);
  split_launch(grid, r->max_grid, [&](int b0, int n, bool, bool last) {
    q.blk0 = b0;
    if (capture)
      hipLaunchKernelGGL(k_sort_scatter<R>, dim3(n), dim3(kSortThreads), 0, st, q);
    else
      hipExtLaunchKernelGGL(k_sort_scatter<R>, dim3(n), dim3(kSortThreads), 0, st, nullptr,
                            last ? e1 : nullptr, 0, q);
  });
  HIP_TRY(hipGetLastError());
  if (!capture) ev_done(r, slot);
  r->pp ^= 1;
  return PIC_OK;
}

template <typename R>
pic_status one_step(pic_run* r, hipStream_t st, bool capture = false) {
  if (r->step > 0 && r->step % r->cfg.sort_interval == 0) {
    pic_status ps = launch_sort<R>(r, st, capture);
    if (ps) return ps;
  }
  pic_status ps = launch_push<R>(r, st, capture);
  if (ps) return ps;
  return launch_field<R>(r, st, capture);
}

// Longest stretch (two sort intervals) replayed as one graph; runs that sort
// more rarely step launch by launch.
constexpr int64_t kMaxGraphSteps = 1024;

void drop_step_graphs(pic_run* r) {
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      if (r->step_graph[a][b]) (void)hipGraphExecDestroy(r->step_graph[a][b]);
      if (r->step_graph_def[a][b]) (void)hipGraphDestroy(r->step_graph_def[a][b]);
      r->step_graph[a][b] = nullptr;
      r->step_graph_def[a][b] = nullptr;
    }
}

// Record the 2 sort_interval steps from the current (sort) step into a graph
// for (pp, step parity); the host's step and sort parity advance as the
// recording does, exactly as the replay will on the device.
template <typename R>
pic_status capture_steps(pic_run* r, int64_t span) {
  if (!r->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&r->capture_stream, hipStreamNonBlocking));
  const int pp = r->pp, fp = (int)(r->step & 1);
  HIP_TRY(hipStreamBeginCapture(r->capture_stream, hipStreamCaptureModeThreadLocal));
  pic_status ps = PIC_OK;
  for (int64_t k = 0; k < span && !ps; ++k) ps = one_step<R>(r, r->capture_stream, true);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(r->capture_stream, &g);
  if (ps) {
    if (g) (void)hipGraphDestroy(g);
    return ps;
  }
  if (e != hipSuccess) return fail(PIC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(PIC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  r->step_graph_def[pp][fp] = g;
  r->step_graph[pp][fp] = x;
  r->step -= span;  // the recording advanced the host state; the launch does it again
  r->pp = pp;
  return PIC_OK;
}

template <typename R>
pic_status do_steps(pic_run* r, int64_t n, hipStream_t st) {
  const int64_t span = 2 * (int64_t)r->cfg.sort_interval;
  while (n > 0) {
    const bool at_sort = r->step > 0 && r->step % r->cfg.sort_interval == 0;
    if (at_sort && !r->timing && span <= kMaxGraphSteps && n >= span) {
      const int pp = r->pp, fp = (int)(r->step & 1);
      if (!r->step_graph[pp][fp]) {
        pic_status ps = capture_steps<R>(r, span);
        if (ps) return ps;
      }
      for (; n >= span; n -= span) {
        HIP_TRY(hipGraphLaunch(r->step_graph[pp][fp], st));
        r->step += span;  // two sorts: the sort parity is back where it was
      }
      continue;
    }
    pic_status ps = one_step<R>(r, st);
    if (ps) return ps;
    --n;
  }
  return PIC_OK;
}

template <typename R>
pic_status do_init(pic_run* r, hipStream_t st) {
  const Derived& d = r->d;
  const long long n = d.n_foil;
  if (n > 0) {
    const int blocks = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_init<R>, dim3(blocks), dim3(256), 0, st, dev<R>(r->sp[0][0]),
                       dev<R>(r->sp[1][0]), n, d.c0, r->cfg.ppc,
                       (unsigned long long)r->cfg.seed, r->cfg.jitter, (R)d.w_ref);
  }
  hipLaunchKernelGGL(k_set_counts, dim3(1), dim3(1), 0, st, r->count, n, n);
  HIP_TRY(hipGetLastError());
  return PIC_OK;
}

// Total field energy and the residual of the energy balance (Section 2):
// what is in the box, plus what was radiated or left it, minus what entered.
void finish_balance(pic_diag_out* o) {
  o->U_field = o->U_Ex + o->U_Et + o->U_B;
  o->balance = o->U_field + o->K_e + o->K_i + o->E_rad + o->E_out_left + o->E_out_right + o->E_esc -
               o->E_in;
}

template <typename R>
pic_status do_diag(pic_run* r, pic_diag_out* out, hipStream_t st) {
  const Derived& d = r->d;
  DiagArgs<R> p{};
  for (int s = 0; s < 2; ++s) p.sp[s] = dev<R>(r->sp[s][r->pp]);
  p.count = r->count + 2 * r->pp;
  p.f = fdev<R>(r, (int)(r->step & 1));
  p.Ex_int = r->Ex_int;
  p.rho = r->rho;
  p.part = r->part;
  p.ipart = r->ipart;
  p.nx = d.nx;
  p.mass[0] = 1.0;
  p.mass[1] = r->cfg.mass_ratio;
  p.Z[0] = -1;
  p.Z[1] = 1;
  p.sw = (R)(256.0 / d.w_ref);
  p.dx = d.dx;
  HIP_TRY(hipMemsetAsync(r->rho, 0, sizeof(long long) * (d.nx + 3), st));
  hipLaunchKernelGGL(k_diag_particles<R>, dim3(2 * kDiagPartBlocks), dim3(kDiagThreads), 0, st, p);
  hipLaunchKernelGGL(k_diag_fields<R>, dim3(kDiagFieldBlocks), dim3(kDiagThreads), 0, st, p);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, st, r->part, r->ipart, r->acc,
                     r->tiles_max, r->dout);
  HIP_TRY(hipGetLastError());
  DiagOutDev o;
  double budget[4];
  int flags[4];
  long long step_dev = 0;
  HIP_TRY(hipMemcpyAsync(&o, r->dout, sizeof(o), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(budget, r->budget, sizeof(budget), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(flags, r->flags, sizeof(flags), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&step_dev, r->step_dev, sizeof(step_dev), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::memset(out, 0, sizeof(*out));
  out->step = r->step;
  out->t = r->step * d.dt;
  out->n_alive[0] = o.alive0;
  out->n_alive[1] = o.alive1;
  out->U_Ex = o.U_Ex;
  out->U_Et = o.U_Et;
  out->U_B = o.U_B;
  out->K_e = o.K_e;
  out->K_i = o.K_i;
  out->E_rad = o.E_rad;
  out->E_in = budget[0];
  out->E_out_left = budget[1];
  out->E_out_right = budget[2];
  out->E_esc = o.E_esc;
  out->gauss_int = o.gauss_int;
  out->gauss = (double)o.gauss_int * d.w_ref * std::ldexp(1.0, -32) / d.dx;
  out->n_stiff = (int64_t)o.n_stiff;
  out->nonfinite = flags[0] != 0;
  finish_balance(out);
  if (step_dev != r->step)
    return fail(PIC_EHIP, "device step counter disagrees with the host (lost launch?)");
  if (out->nonfinite) return fail(PIC_ENONFINITE, "a particle momentum became non-finite");
  return PIC_OK;
}

size_t rsz(const pic_run* r) { return r->d.rsize; }


// ---------------------------------------------------------------- batches
size_t slot_bytes_for(int prec) {
  return prec == PIC_FP32 ? sizeof(SlotDev<float>) : sizeof(SlotDev<double>);
}

}  // namespace

struct pic_batch {
  int prec;
  int max_slots, quantum;
  int cap[3];                 // work-group capacity: push, field, sort
  char* tab;                  // device slot table
  size_t slot_bytes;
  // device work ranges [max_slots + 1]: push tiles, field chunks, sort
  // tiles, field chunks of the persistent launch (kThreads nodes)
  int* start[4];
  long long* dummy_step;      // step counter of free slots
  long long* steps;           // [max_slots] gathered step counters
  int* done;                  // [max_slots][kDoneStride] field chunks finished this step
  unsigned* bar;              // grid barrier words of the persistent launch
  int* err;                   // set by a persistent launch whose barrier timed out
  std::vector<pic_run*> runs;
  std::vector<long long> target;
  std::vector<int> nblk[4];
  bool persistent = false;    // steps of a quantum in one launch (else one launch per pass)
  unsigned long long bar_ticks = kBarTicks;  // longest grid-barrier wait of the persistent launch
  int persist_cap = 0;        // work-groups of the persistent launch that fit the device at once
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // captured kernel nodes whose grid follows the resident work: kind 0 push,
  // 1 field, 2 sort (hist and scatter), 3 persistent steps
  std::vector<std::pair<hipGraphNode_t, int>> nodes;
  // asynchronous poll: step counters and the error word land in pinned host
  // memory behind the queued replays; a slot whose run changed since the
  // poll was queued (admit or release bump its generation) reads -1
  long long* pin_steps = nullptr;  // [max_slots + 1], the last entry the error word
  hipEvent_t poll_ev = nullptr;
  bool poll_pending = false;
  std::vector<unsigned long long> gen, gen_snap;
};

namespace {

size_t batch_layout(int prec, int max_slots, pic_batch* b, char* base) {
  Carver cv{base};
  char* tab = cv.take<char>(slot_bytes_for(prec) * max_slots);
  int* st[4];
  for (int k = 0; k < 4; ++k) st[k] = cv.take<int>(max_slots + 1);
  long long* dummy = cv.take<long long>(1);
  long long* steps = cv.take<long long>(max_slots);
  int* done = cv.take<int>((size_t)kDoneStride * max_slots);
  unsigned* bar = cv.take<unsigned>(kBarWords);
  int* err = cv.take<int>(32);
  if (b) {
    b->tab = tab;
    for (int k = 0; k < 4; ++k) b->start[k] = st[k];
    b->dummy_step = dummy;
    b->steps = steps;
    b->done = done;
    b->bar = bar;
    b->err = err;
  }
  return cv.off + 256;
}

template <typename R>
SlotDev<R> make_slot(const pic_batch* b, int slot, const pic_run* r, long long target) {
  SlotDev<R> e{};
  e.done = b->done + (size_t)kDoneStride * slot;
  if (!r) {
    e.step = b->dummy_step;
    e.target = 0;
    e.sort_interval = b->quantum;
    return e;
  }
  for (int pp = 0; pp < 2; ++pp)
    for (int fp = 0; fp < 2; ++fp) e.push[pp][fp] = make_push_args<R>(r, pp, fp, kBatchTile);
  for (int fp = 0; fp < 2; ++fp) e.field[fp] = make_field_args<R>(r, fp, 0);
  for (int q = 0; q < 2; ++q) e.sort[q] = make_sort_args<R>(r, q);
  for (int s = 0; s < 2; ++s) {
    e.cnt[s] = r->cnt[s];
    e.cur[s] = r->cursor[s];
  }
  e.count = r->count;
  e.step = r->step_dev;
  e.target = target;
  e.sort_interval = r->cfg.sort_interval;
  e.nx = r->d.nx;
  return e;
}

template <typename R>
pic_status write_slot(pic_batch* b, int slot, hipStream_t st) {
  const SlotDev<R> e = make_slot<R>(b, slot, b->runs[slot], b->target[slot]);
  HIP_TRY(hipMemcpyAsync(b->tab + slot * b->slot_bytes, &e, sizeof(e), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return PIC_OK;
}

pic_status update_batch_grids(pic_batch* b);

pic_status write_ranges(pic_batch* b, hipStream_t st) {
  std::vector<int> h((size_t)4 * (b->max_slots + 1));
  for (int k = 0; k < 4; ++k) {
    int* o = h.data() + k * (b->max_slots + 1);
    o[0] = 0;
    for (int s = 0; s < b->max_slots; ++s) o[s + 1] = o[s] + b->nblk[k][s];
    HIP_TRY(hipMemcpyAsync(b->start[k], o, (b->max_slots + 1) * sizeof(int), hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  return update_batch_grids(b);
}

// Work-groups a run of n0 electrons, n1 ions and nx cells occupies in each
// captured launch of a batch: push tiles, field chunks, sort tiles, and the
// field chunks of the persistent launch (no capacity: they follow nx).
void batch_need(long long n0, long long n1, int nx, int need[4]) {
  need[0] = tiles_for(n0, kBatchTile) + tiles_for(n1, kBatchTile);
  need[1] = (nx + 3 + kFieldChunk - 1) / kFieldChunk;
  need[2] = sort_blocks_for(n0) + sort_blocks_for(n1);
  need[3] = (nx + 3 + kThreads - 1) / kThreads;
}

// The resident runs leave room for `need`.
bool batch_room(const pic_batch* b, const int need[3]) {
  for (int k = 0; k < 3; ++k) {
    long long used = 0;
    for (int s = 0; s < b->max_slots; ++s) used += b->nblk[k][s];
    if (used + need[k] > b->cap[k]) return false;
  }
  return true;
}

int batch_work(const pic_batch* b, int kind) {
  long long t = 0;
  for (int s = 0; s < b->max_slots; ++s) t += b->nblk[kind][s];
  return (int)std::max<long long>(1, t);
}

template <typename R>
pic_status capture_batch(pic_batch* b, hipStream_t st) {
  const SlotDev<R>* tab = reinterpret_cast<const SlotDev<R>*>(b->tab);
  const int n = b->max_slots;
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (b->persistent) {
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_steps_batch<R>, kThreads, 0));
    if (per_cu < 1) return fail(PIC_EHIP, "persistent batch kernel does not fit a compute unit");
    if (PIC_STEPS_BLOCKS_PER_CU > 0) per_cu = std::min(per_cu, PIC_STEPS_BLOCKS_PER_CU);
    b->persist_cap = per_cu * cus;
  }
  HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
  // every admitted run is at a multiple of the quantum here, so the sort
  // (when due) is the first stage of the quantum; grids are set to the
  // resident work (one work-group per tile) by update_batch_grids
  hipLaunchKernelGGL(k_sort_hist_batch<R>, dim3(1), dim3(kSortThreads), 0, st, tab, b->start[2], n);
  hipLaunchKernelGGL(k_sort_scan_batch<R>, dim3(std::min(2 * n, cus)), dim3(1024), 0, st, tab, n);
  hipLaunchKernelGGL(k_sort_scatter_batch<R>, dim3(1), dim3(kSortThreads), 0, st, tab, b->start[2], n);
  if (b->persistent) {
    hipLaunchKernelGGL(k_steps_batch<R>, dim3(1), dim3(kThreads), 0, st, tab, b->start[0], b->start[3], n,
                       b->quantum, b->bar, b->err, b->bar_ticks);
  } else {
    for (int q = 0; q < b->quantum; ++q) {
      hipLaunchKernelGGL(k_push_batch<R>, dim3(1), dim3(kThreads), 0, st, tab, b->start[0], n);
      hipLaunchKernelGGL(k_field_batch<R>, dim3(1), dim3(kFieldChunk), 0, st, tab, b->start[1], n);
    }
  }
  hipError_t e = hipStreamEndCapture(st, &b->graph);
  if (e != hipSuccess) return fail(PIC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  // remember the nodes whose grid follows the work
  size_t num = 0;
  HIP_TRY(hipGraphGetNodes(b->graph, nullptr, &num));
  std::vector<hipGraphNode_t> all(num);
  HIP_TRY(hipGraphGetNodes(b->graph, all.data(), &num));
  const void* fpush = reinterpret_cast<const void*>(&k_push_batch<R>);
  const void* ffield = reinterpret_cast<const void*>(&k_field_batch<R>);
  const void* fhist = reinterpret_cast<const void*>(&k_sort_hist_batch<R>);
  const void* fscat = reinterpret_cast<const void*>(&k_sort_scatter_batch<R>);
  const void* fsteps = reinterpret_cast<const void*>(&k_steps_batch<R>);
  b->nodes.clear();
  for (hipGraphNode_t nd : all) {
    hipGraphNodeType ty;
    HIP_TRY(hipGraphNodeGetType(nd, &ty));
    if (ty != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams kp{};
    HIP_TRY(hipGraphKernelNodeGetParams(nd, &kp));
    const int kind = kp.func == fpush ? 0 : kp.func == ffield ? 1 : (kp.func == fhist || kp.func == fscat) ? 2
                     : kp.func == fsteps ? 3 : -1;
    if (kind >= 0) b->nodes.emplace_back(nd, kind);
  }
  return PIC_OK;
}

// Set the grids of the captured launches to the resident work.
pic_status update_batch_grids(pic_batch* b) {
  if (!b->exec) return PIC_OK;
  // the persistent launch: enough work-groups for the larger pass, no more
  // than fit the device at once (its barriers need every one resident)
  const int work[4] = {batch_work(b, 0), batch_work(b, 1), batch_work(b, 2),
                       std::min(b->persist_cap, std::max(batch_work(b, 0), batch_work(b, 3)))};
  for (auto& nk : b->nodes) {
    hipKernelNodeParams kp{};
    HIP_TRY(hipGraphKernelNodeGetParams(nk.first, &kp));
    kp.gridDim = dim3(work[nk.second]);
    HIP_TRY(hipGraphExecKernelNodeSetParams(b->exec, nk.first, &kp));
  }
  return PIC_OK;
}

__global__ void k_gather_steps(const char* tab, size_t slot_bytes, size_t step_off, int n,
                               long long* out) {
  const int s = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (s < n) out[s] = **reinterpret_cast<long long* const*>(tab + s * slot_bytes + step_off);
}

// ---------------------------------------------------------------- static scratch
__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) p[i] = v;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's copy of `scratch`, looked up once per device with
// that device current (every device has its own copy at its own address).
pic_status static_scratch(unsigned long long** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PIC_EINVAL, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(PIC_EHIP, "hipGetSymbolAddress returned a null address");
    g_scratch_ptr[dev] = static_cast<unsigned long long*>(p);
  }
  *out = g_scratch_ptr[dev];
  return PIC_OK;
}

// ---------------------------------------------------------------- checkpointed budget
// The per-tile accumulators hold, per push work-group slot, the radiated
// energy, the escaped energy of each species and the stiff-push count.
// A checkpoint carries their totals; a restore puts the totals in slot 0 and
// clears the rest, so the run's sums continue from them.
pic_status read_tile_budget(const double* acc, int tiles, const int* flags, pic_budget_state* b) {
  std::vector<double> a(4 * (size_t)std::max(tiles, 1));
  HIP_TRY(hipMemcpy(a.data(), acc, a.size() * sizeof(double), hipMemcpyDeviceToHost));
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  for (size_t i = 0; i < a.size(); ++i) t[i % 4] += a[i];
  b->E_rad = t[0];
  b->E_esc[0] = t[1];
  b->E_esc[1] = t[2];
  b->n_stiff = t[3];
  int f = 0;
  HIP_TRY(hipMemcpy(&f, flags, sizeof(int), hipMemcpyDeviceToHost));
  b->nonfinite = f != 0;
  b->valid = 1;
  return PIC_OK;
}

pic_status write_tile_budget(double* acc, int tiles, int* flags, const pic_budget_state* b) {
  std::vector<double> a(4 * (size_t)std::max(tiles, 1), 0.0);
  a[0] = b->E_rad;
  a[1] = b->E_esc[0];
  a[2] = b->E_esc[1];
  a[3] = b->n_stiff;
  HIP_TRY(hipMemcpy(acc, a.data(), a.size() * sizeof(double), hipMemcpyHostToDevice));
  const int f = b->nonfinite ? 1 : 0;
  HIP_TRY(hipMemcpy(flags, &f, sizeof(int), hipMemcpyHostToDevice));
  return PIC_OK;
}


}  // namespace

extern "C" {

const char* pic_last_error(void) { return g_err.c_str(); }

pic_status pic_workspace_bytes(const pic_config* cfg, size_t* bytes) {
  if (!bytes) return fail(PIC_EINVAL, "null bytes pointer");
  pic_run tmp;
  // validate (null config, struct_size of the caller's layout) before copying it
  pic_status st = derive(cfg, &tmp.d);
  if (st) return st;
  tmp.cfg = *cfg;
  Carver cv{nullptr};
  carve(&tmp, cv);
  *bytes = cv.off + 256;
  return PIC_OK;
}

pic_status pic_init(const pic_config* cfg, void* d_ws, size_t ws_bytes, void* stream,
                    pic_run** out) {
  if (!out) return fail(PIC_EINVAL, "null output handle");
  *out = nullptr;
  if (!d_ws) return fail(PIC_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256)
    return fail(PIC_EINVAL, "workspace must be 256-byte aligned");
  size_t need = 0;
  pic_status st = pic_workspace_bytes(cfg, &need);
  if (st) return st;
  if (ws_bytes < need)
    return fail(PIC_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  pic_run* r = new pic_run();
  r->cfg = *cfg;
  derive(cfg, &r->d);
  Carver cv{static_cast<char*>(d_ws)};
  carve(r, cv);
  r->n_max[0] = r->n_max[1] = r->d.n_foil;
  r->step = 0;
  r->pp = 0;
  // Small runs push in tiles of kBatchTile: with fewer than two large tiles
  // per compute unit the large tiles leave most of the device idle (on
  // 4e5 particles the small tiles push 1.85x faster, on 1e7 the large ones
  // 1.27x).  Fixed for the run: the push's window predictions are per tile.
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        2 * tiles_for(r->d.n_foil) < 2 * cus)  // both species' large tiles
      r->push_tile = kBatchTile;
  }
  hipStream_t s = S(stream);
  hipError_t e = hipMemsetAsync(d_ws, 0, cv.off, s);
  if (e != hipSuccess) {
    delete r;
    return fail(PIC_EHIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
  }
  st = r->d.prec == PIC_FP32 ? do_init<float>(r, s) : do_init<double>(r, s);
  if (st) {
    delete r;
    return st;
  }
  *out = r;
  return PIC_OK;
}

pic_status pic_step(pic_run* r, int64_t n, void* stream) {
  if (!r || n < 0) return fail(PIC_EINVAL, "null run or negative step count");
  if (r->batch) return fail(PIC_EBUSY, "run is stepped by a batch; release it first");
  return r->d.prec == PIC_FP32 ? do_steps<float>(r, n, S(stream)) : do_steps<double>(r, n, S(stream));
}

pic_status pic_push_deposit(pic_run* r, void* stream) {
  if (!r) return fail(PIC_EINVAL, "null run");
  if (r->batch) return fail(PIC_EBUSY, "run is stepped by a batch; release it first");
  return r->d.prec == PIC_FP32 ? launch_push<float>(r, S(stream)) : launch_push<double>(r, S(stream));
}

pic_status pic_field_advance(pic_run* r, void* stream) {
  if (!r) return fail(PIC_EINVAL, "null run");
  if (r->batch) return fail(PIC_EBUSY, "run is stepped by a batch; release it first");
  return r->d.prec == PIC_FP32 ? launch_field<float>(r, S(stream)) : launch_field<double>(r, S(stream));
}

pic_status pic_sort(pic_run* r, void* stream) {
  if (!r) return fail(PIC_EINVAL, "null run");
  if (r->batch) return fail(PIC_EBUSY, "run is stepped by a batch; release it first");
  return r->d.prec == PIC_FP32 ? launch_sort<float>(r, S(stream)) : launch_sort<double>(r, S(stream));
}

pic_status pic_diag(pic_run* r, pic_diag_out* out, void* stream) {
  if (!r || !out) return fail(PIC_EINVAL, "null run or output");
  if (r->batch) return fail(PIC_EBUSY, "run is stepped by a batch; release it first");
  return r->d.prec == PIC_FP32 ? do_diag<float>(r, out, S(stream)) : do_diag<double>(r, out, S(stream));
}

pic_status pic_get_info(const pic_run* r, pic_info* o) {
  if (!r || !o) return fail(PIC_EINVAL, "null run or output");
  o->n_cells = r->d.nx;
  o->precision = r->d.prec;
  o->dx = r->d.dx;
  o->dt = r->d.dt;
  o->eps_rr = r->d.eps;
  o->w_ref = r->d.w_ref;
  o->capacity = r->d.cap;
  o->n_init[0] = r->n_max[0];
  o->n_init[1] = r->n_max[1];
  o->step = r->step;
  o->tile = r->push_tile;
  o->lds_slots = kLdsSlots;
  return PIC_OK;
}

void pic_free(pic_run* r) {
  if (!r || r->batch) return;
  for (auto& e : r->ev) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  drop_step_graphs(r);
  if (r->capture_stream) (void)hipStreamDestroy(r->capture_stream);
  delete r;
}

pic_status pic_get_particles(pic_run* r, int32_t species, int64_t first, int64_t count,
                             pic_species_state* o, void* stream) {
  if (!r || !o) return fail(PIC_EINVAL, "null run or output");
  if (r->batch) return fail(PIC_EBUSY, "run is stepped by a batch; release it first");
  if (species != 0 && species != 1) return fail(PIC_EINVAL, "species must be 0 or 1");
  if (first < 0 || count < 0) return fail(PIC_EINVAL, "negative range");
  hipStream_t s = S(stream);
  HIP_TRY(hipStreamSynchronize(s));
  long long n = 0;
  HIP_TRY(hipMemcpy(&n, r->count + 2 * r->pp + species, sizeof(n), hipMemcpyDeviceToHost));
  const long long m = std::max(0ll, std::min<long long>(count, n - first));
  o->count = m;
  if (!m) return PIC_OK;
  const SpeciesBuf& b = r->sp[species][r->pp];
  const size_t rs = rsz(r);
  auto pull = [&](void* dst, const void* src, size_t es) -> pic_status {
    if (!dst || !src) return PIC_OK;
    HIP_TRY(hipMemcpy(dst, static_cast<const char*>(src) + first * es, m * es, hipMemcpyDeviceToHost));
    return PIC_OK;
  };
  pic_status ps;
  if ((ps = pull(o->cell, b.cell, 4)) || (ps = pull(o->off, b.off, rs)) || (ps = pull(o->ux, b.ux, rs)) ||
      (ps = pull(o->uy, b.uy, rs)) || (ps = pull(o->uz, b.uz, rs)) || (ps = pull(o->w, b.w, rs)) ||
      (ps = pull(o->rx, b.rx, 4)) || (ps = pull(o->ry, b.ry, 4)) || (ps = pull(o->rz, b.rz, 4)))
    return ps;
  return PIC_OK;
}

pic_status pic_get_state(pic_run* r, pic_state* st, void* stream) {
  if (!r || !st) return fail(PIC_EINVAL, "null run or state");
  if (r->batch) return fail(PIC_EBUSY, "run is stepped by a batch; release it first");
  hipStream_t s = S(stream);
  const Derived& d = r->d;
  const size_t rs = rsz(r);
  HIP_TRY(hipStreamSynchronize(s));
  long long cnt[2];
  HIP_TRY(hipMemcpy(cnt, r->count + 2 * r->pp, sizeof(cnt), hipMemcpyDeviceToHost));
  for (int sp = 0; sp < 2; ++sp) {
    pic_species_state& o = st->sp[sp];
    const SpeciesBuf& b = r->sp[sp][r->pp];
    const long long n = cnt[sp];
    if (!o.cell && !o.off && !o.ux && !o.uy && !o.uz && !o.w && !o.rx && !o.ry && !o.rz) {
      o.count = 0;  // fields only
      continue;
    }
    std::vector<int> cell(n);
    if (n) HIP_TRY(hipMemcpy(cell.data(), b.cell, n * sizeof(int), hipMemcpyDeviceToHost));
    std::vector<long long> idx;
    idx.reserve(n);
    for (long long i = 0; i < n; ++i)
      if (cell[i] != kDead) idx.push_back(i);
    o.count = (int64_t)idx.size();
    if (o.cell)
      for (size_t k = 0; k < idx.size(); ++k) o.cell[k] = cell[idx[k]];
    auto pull = [&](void* dst, const void* src, size_t es) -> pic_status {
      if (!dst || !src) return PIC_OK;
      std::vector<char> tmp(n * es);
      if (n) HIP_TRY(hipMemcpy(tmp.data(), src, n * es, hipMemcpyDeviceToHost));
      for (size_t k = 0; k < idx.size(); ++k)
        std::memcpy(static_cast<char*>(dst) + k * es, tmp.data() + idx[k] * es, es);
      return PIC_OK;
    };
    pic_status ps;
    if ((ps = pull(o.off, b.off, rs)) || (ps = pull(o.ux, b.ux, rs)) || (ps = pull(o.uy, b.uy, rs)) ||
        (ps = pull(o.uz, b.uz, rs)) || (ps = pull(o.w, b.w, rs)) || (ps = pull(o.rx, b.rx, 4)) ||
        (ps = pull(o.ry, b.ry, 4)) || (ps = pull(o.rz, b.rz, 4)))
      return ps;
  }
  {  // de-interleave the fields of the current step
    const int p = (int)(r->step & 1);
    std::vector<char> nb((size_t)(d.nx + 1) * 2 * rs), hb((size_t)(d.nx + 2) * 4 * rs);
    HIP_TRY(hipMemcpy(nb.data(), r->FN[p], nb.size(), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hb.data(), r->FH[p], hb.size(), hipMemcpyDeviceToHost));
    void* outs[5] = {st->Ex, st->Ey, st->Ez, st->By, st->Bz};
    for (int k = 0; k < 5; ++k) {
      if (!outs[k]) continue;
      const bool node = (k == 1 || k == 2);
      const size_t len = node ? d.nx + 1 : d.nx + 2, stride = node ? 2 : 4;
      const size_t comp = k == 0 ? 0 : k == 1 ? 0 : k == 2 ? 1 : k == 3 ? 1 : 2;
      const char* src = node ? nb.data() : hb.data();
      for (size_t i = 0; i < len; ++i)
        std::memcpy(static_cast<char*>(outs[k]) + i * rs, src + (i * stride + comp) * rs, rs);
    }
  }
  if (st->Ex_int)
    HIP_TRY(hipMemcpy(st->Ex_int, r->Ex_int, (d.nx + 2) * sizeof(long long), hipMemcpyDeviceToHost));
  int64_t* js[3] = {st->Jx_int, st->Jy_int, st->Jz_int};
  const size_t jl[3] = {(size_t)d.nx + 2, (size_t)d.nx + 3, (size_t)d.nx + 3};
  for (int k = 0; k < 3; ++k)
    if (js[k])
      HIP_TRY(hipMemcpy(js[k], r->J[r->step & 1][k], jl[k] * sizeof(long long), hipMemcpyDeviceToHost));
  st->step = r->step;
  {
    double bud[4];
    HIP_TRY(hipMemcpy(bud, r->budget, sizeof(bud), hipMemcpyDeviceToHost));
    st->budget.E_in = bud[0];
    st->budget.E_out_left = bud[1];
    st->budget.E_out_right = bud[2];
    pic_status ps = read_tile_budget(r->acc, r->tiles_max, r->flags, &st->budget);
    if (ps) return ps;
  }
  return PIC_OK;
}

pic_status pic_set_state(pic_run* r, const pic_state* st, void* stream) {
  if (!r || !st) return fail(PIC_EINVAL, "null run or state");
  if (r->batch) return fail(PIC_EBUSY, "run is stepped by a batch; release it first");
  hipStream_t s = S(stream);
  const Derived& d = r->d;
  const size_t rs = rsz(r);
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemset(r->tpred, 0, 2 * sizeof(int)));  // the tile ranges no longer hold
  drop_step_graphs(r);  // particle counts (launch grids) may change
  if (st->step >= 0 && st->step != r->step) {
    // move the fields to the buffer parity of the new step
    const int po = (int)(r->step & 1), pn = (int)(st->step & 1);
    if (po != pn) {
      HIP_TRY(hipMemcpy(r->FN[pn], r->FN[po], (size_t)(d.nx + 1) * 2 * rs, hipMemcpyDeviceToDevice));
      HIP_TRY(hipMemcpy(r->FH[pn], r->FH[po], (size_t)(d.nx + 2) * 4 * rs, hipMemcpyDeviceToDevice));
    }
    r->step = st->step;
    HIP_TRY(hipMemcpy(r->step_dev, &r->step, sizeof(long long), hipMemcpyHostToDevice));
  }
  for (int sp = 0; sp < 2; ++sp) {
    const pic_species_state& o = st->sp[sp];
    const bool any = o.cell || o.off || o.ux || o.uy || o.uz || o.w;
    if (!any) continue;
    if (!(o.cell && o.off && o.ux && o.uy && o.uz && o.w))
      return fail(PIC_EINVAL, "particle arrays must be all given or all null");
    if (o.count < 0 || o.count > d.cap) return fail(PIC_ENOMEM, "particle count exceeds capacity");
    const long long n = o.count;
    for (long long i = 0; i < n; ++i) {
      const double off = rs == 4 ? (double)static_cast<const float*>(o.off)[i]
                                 : static_cast<const double*>(o.off)[i];
      if (o.cell[i] < 0 || o.cell[i] >= d.nx || !(off >= 0.0 && off < 1.0))
        return fail(PIC_EINVAL, "particle " + std::to_string(i) + " of species " +
                                    std::to_string(sp) + " has cell/offset out of range");
    }
    const SpeciesBuf& b = r->sp[sp][r->pp];
    if (n) {
      HIP_TRY(hipMemcpy(b.cell, o.cell, n * sizeof(int), hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(b.off, o.off, n * rs, hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(b.ux, o.ux, n * rs, hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(b.uy, o.uy, n * rs, hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(b.uz, o.uz, n * rs, hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(b.w, o.w, n * rs, hipMemcpyHostToDevice));
      if (b.rx) {
        if (o.rx && o.ry && o.rz) {
          HIP_TRY(hipMemcpy(b.rx, o.rx, n * 4, hipMemcpyHostToDevice));
          HIP_TRY(hipMemcpy(b.ry, o.ry, n * 4, hipMemcpyHostToDevice));
          HIP_TRY(hipMemcpy(b.rz, o.rz, n * 4, hipMemcpyHostToDevice));
        } else {
          HIP_TRY(hipMemset(b.rx, 0, n * 4));
          HIP_TRY(hipMemset(b.ry, 0, n * 4));
          HIP_TRY(hipMemset(b.rz, 0, n * 4));
        }
      }
    }
    HIP_TRY(hipMemcpy(r->count + 2 * r->pp + sp, &n, sizeof(long long), hipMemcpyHostToDevice));
    r->n_max[sp] = n;
    for (int p = 0; p < 2; ++p)
      for (int k = 0; k < 3; ++k) HIP_TRY(hipMemset(r->J[p][k], 0, (d.nx + 3) * sizeof(long long)));
  }
  {  // interleave the given fields into the current step's buffers
    const int p = (int)(r->step & 1);
    const void* ins[5] = {st->Ex, st->Ey, st->Ez, st->By, st->Bz};
    if (ins[0] || ins[1] || ins[2] || ins[3] || ins[4]) {
      std::vector<char> nb((size_t)(d.nx + 1) * 2 * rs), hb((size_t)(d.nx + 2) * 4 * rs);
      HIP_TRY(hipMemcpy(nb.data(), r->FN[p], nb.size(), hipMemcpyDeviceToHost));
      HIP_TRY(hipMemcpy(hb.data(), r->FH[p], hb.size(), hipMemcpyDeviceToHost));
      for (int k = 0; k < 5; ++k) {
        if (!ins[k]) continue;
        const bool node = (k == 1 || k == 2);
        const size_t len = node ? d.nx + 1 : d.nx + 2, stride = node ? 2 : 4;
        const size_t comp = k == 0 ? 0 : k == 1 ? 0 : k == 2 ? 1 : k == 3 ? 1 : 2;
        char* dst = node ? nb.data() : hb.data();
        for (size_t i = 0; i < len; ++i)
          std::memcpy(dst + (i * stride + comp) * rs, static_cast<const char*>(ins[k]) + i * rs, rs);
      }
      HIP_TRY(hipMemcpy(r->FN[p], nb.data(), nb.size(), hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(r->FH[p], hb.data(), hb.size(), hipMemcpyHostToDevice));
    }
  }
  if (st->Ex_int)
    HIP_TRY(hipMemcpy(r->Ex_int, st->Ex_int, (d.nx + 2) * sizeof(long long), hipMemcpyHostToDevice));
  const int64_t* js[3] = {st->Jx_int, st->Jy_int, st->Jz_int};
  const size_t jl[3] = {(size_t)d.nx + 2, (size_t)d.nx + 3, (size_t)d.nx + 3};
  for (int k = 0; k < 3; ++k)
    if (js[k])
      HIP_TRY(hipMemcpy(r->J[r->step & 1][k], js[k], jl[k] * sizeof(long long), hipMemcpyHostToDevice));
  if (st->budget.valid) {
    const double bud[4] = {st->budget.E_in, st->budget.E_out_left, st->budget.E_out_right, 0.0};
    HIP_TRY(hipMemcpy(r->budget, bud, sizeof(bud), hipMemcpyHostToDevice));
    pic_status ps = write_tile_budget(r->acc, r->tiles_max, r->flags, &st->budget);
    if (ps) return ps;
  }
  HIP_TRY(hipDeviceSynchronize());
  return PIC_OK;
}

pic_status pic_spectrum_static(pic_run* r, int32_t bins, double e_max, double* host_hist, void* stream) {
  if (!r || !host_hist || bins < 1 || !(e_max > 0)) return fail(PIC_EINVAL, "bad spectrum arguments");
  if (bins > kStaticSpectrumBins)
    return fail(PIC_EINVAL, "pic_spectrum_static takes at most " + std::to_string(kStaticSpectrumBins) + " bins");
  if (r->batch) return fail(PIC_EBUSY, "run is stepped by a batch; release it first");
  unsigned long long* hist = nullptr;
  pic_status ps = static_scratch(&hist);
  if (ps) return ps;
  hipStream_t s = S(stream);
  // the array keeps the last call's counts: clear the bins this call uses
  hipLaunchKernelGGL(k_fill_u64, dim3((bins + 255) / 256), dim3(256), 0, s, hist, bins, 0ull);
  const double mc2 = r->cfg.mass_ratio * kMec2_MeV;
  if (r->d.prec == PIC_FP32)
    hipLaunchKernelGGL(k_spectrum<float>, dim3(1024), dim3(256), 0, s, dev<float>(r->sp[1][r->pp]),
                       r->count + 2 * r->pp + 1, hist, bins, e_max, mc2, (float)(256.0 / r->d.w_ref));
  else
    hipLaunchKernelGGL(k_spectrum<double>, dim3(1024), dim3(256), 0, s, dev<double>(r->sp[1][r->pp]),
                       r->count + 2 * r->pp + 1, hist, bins, e_max, mc2, 256.0 / r->d.w_ref);
  HIP_TRY(hipGetLastError());
  // the 64-bit counts land in the caller's array and are converted in place
  static_assert(sizeof(double) == sizeof(unsigned long long), "in-place conversion");
  HIP_TRY(hipMemcpyAsync(host_hist, hist, bins * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double de = e_max / bins, unit = r->d.w_ref / 256.0;
  for (int b = 0; b < bins; ++b) {
    long long c;
    std::memcpy(&c, host_hist + b, sizeof(c));
    host_hist[b] = (double)c * unit / de;
  }
  return PIC_OK;
}

pic_status pic_spectrum(pic_run* r, int32_t bins, double e_max, double* host_hist, void* stream) {
  if (!r || !host_hist || bins < 1 || bins > kMaxSpectrumBins || !(e_max > 0))
    return fail(PIC_EINVAL, "bad spectrum arguments");
  hipStream_t s = S(stream);
  const double mc2 = r->cfg.mass_ratio * kMec2_MeV;
  HIP_TRY(hipMemsetAsync(r->hist, 0, bins * sizeof(unsigned long long), s));
  const int blocks = 1024;
  if (r->d.prec == PIC_FP32)
    hipLaunchKernelGGL(k_spectrum<float>, dim3(blocks), dim3(256), 0, s, dev<float>(r->sp[1][r->pp]),
                       r->count + 2 * r->pp + 1, r->hist, bins, e_max, mc2,
                       (float)(256.0 / r->d.w_ref));
  else
    hipLaunchKernelGGL(k_spectrum<double>, dim3(blocks), dim3(256), 0, s, dev<double>(r->sp[1][r->pp]),
                       r->count + 2 * r->pp + 1, r->hist, bins, e_max, mc2, 256.0 / r->d.w_ref);
  HIP_TRY(hipGetLastError());
  std::vector<long long> h(bins);
  HIP_TRY(hipMemcpyAsync(h.data(), r->hist, bins * sizeof(long long), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double de = e_max / bins, unit = r->d.w_ref / 256.0;
  for (int b = 0; b < bins; ++b) host_hist[b] = (double)h[b] * unit / de;
  return PIC_OK;
}

pic_status pic_friction(pic_run* r, int32_t bins, double log10_lo, double log10_hi, double* host_hist,
                        double* host_stats, void* stream) {
  if (!r || !host_hist || !host_stats || bins < 1 || bins > kMaxSpectrumBins - 5 ||
      !(log10_hi > log10_lo) || !std::isfinite(log10_lo) || !std::isfinite(log10_hi))
    return fail(PIC_EINVAL, "bad friction arguments");
  if (r->batch) return fail(PIC_EBUSY, "run is stepped by a batch; release it first");
  hipStream_t s = S(stream);
  double* out = reinterpret_cast<double*>(r->hist);  // the spectrum's counters, as FP64 sums
  HIP_TRY(hipMemsetAsync(out, 0, (bins + 5) * sizeof(double), s));
  const int p = (int)(r->step & 1);
  if (r->d.prec == PIC_FP32)
    hipLaunchKernelGGL(k_friction<float>, dim3(1024), dim3(256), 0, s, dev<float>(r->sp[0][r->pp]),
                       fdev<float>(r, p), r->count + 2 * r->pp, out, bins, log10_lo, log10_hi, r->d.eps);
  else
    hipLaunchKernelGGL(k_friction<double>, dim3(1024), dim3(256), 0, s, dev<double>(r->sp[0][r->pp]),
                       fdev<double>(r, p), r->count + 2 * r->pp, out, bins, log10_lo, log10_hi, r->d.eps);
  HIP_TRY(hipGetLastError());
  std::vector<double> h(bins + 5);
  HIP_TRY(hipMemcpyAsync(h.data(), out, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int b = 0; b < bins; ++b) host_hist[b] = h[b];
  host_stats[0] = h[bins + 2];
  host_stats[1] = h[bins + 4] > 0 ? h[bins + 3] / h[bins + 4] : 0.0;
  host_stats[2] = h[bins];
  host_stats[3] = h[bins + 1];
  return PIC_OK;
}

pic_status pic_track(const pic_wave* wave, int32_t scheme, int32_t rr, int32_t precision,
                     double lambda_um, double dt, double t0, int64_t steps, int64_t n, double* d_x,
                     double* d_ux, double* d_uy, double* d_uz, void* stream) {
  if (!wave) return fail(PIC_EINVAL, "null wave");
  if (scheme != PIC_TRACK_LEAPFROG && scheme != PIC_TRACK_RK4) return fail(PIC_EINVAL, "unknown scheme");
  if (rr != PIC_RR_OFF && rr != PIC_RR_REDUCED && rr != PIC_RR_FULL) return fail(PIC_EINVAL, "unknown rr mode");
  if (precision != PIC_FP32 && precision != PIC_FP64) return fail(PIC_EINVAL, "bad precision");
  if (!(lambda_um > 0.0) || !(dt > 0.0) || steps < 0 || n < 0 || !std::isfinite(t0))
    return fail(PIC_EINVAL, "bad wavelength, step, count or start time");
  if (!std::isfinite(wave->a_y) || !std::isfinite(wave->a_z) || !std::isfinite(wave->psi))
    return fail(PIC_EINVAL, "non-finite wave parameters");
  if (n > 0 && (!d_x || !d_ux || !d_uy || !d_uz)) return fail(PIC_EINVAL, "null particle arrays");
  if (n == 0 || steps == 0) return PIC_OK;
  TrackArgs a{};
  a.ay = wave->a_y;
  a.az = wave->a_z;
  a.psi = wave->psi;
  a.dt = dt;
  a.t0 = t0;
  a.eps = 4.0 * M_PI / 3.0 * kRe_um / lambda_um;
  a.steps = steps;
  a.n = n;
  a.x = d_x;
  a.ux = d_ux;
  a.uy = d_uy;
  a.uz = d_uz;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  hipStream_t st = S(stream);
  const bool f32 = precision == PIC_FP32;
#define PIC_TRACK_LAUNCH(K, M)                                                      \
  do {                                                                              \
    if (f32)                                                                        \
      hipLaunchKernelGGL((K<float, M>), grid, block, 0, st, a);                     \
    else                                                                            \
      hipLaunchKernelGGL((K<double, M>), grid, block, 0, st, a);                    \
  } while (0)
  if (scheme == PIC_TRACK_LEAPFROG) {
    if (rr == PIC_RR_OFF) PIC_TRACK_LAUNCH(k_track_leapfrog, 0);
    else if (rr == PIC_RR_REDUCED) PIC_TRACK_LAUNCH(k_track_leapfrog, 1);
    else PIC_TRACK_LAUNCH(k_track_leapfrog, 2);
  } else {
    if (rr == PIC_RR_OFF) PIC_TRACK_LAUNCH(k_track_rk4, 0);
    else if (rr == PIC_RR_REDUCED) PIC_TRACK_LAUNCH(k_track_rk4, 1);
    else PIC_TRACK_LAUNCH(k_track_rk4, 2);
  }
#undef PIC_TRACK_LAUNCH
  HIP_TRY(hipGetLastError());
  return PIC_OK;
}

pic_status pic_check_rounding(uint32_t first, uint32_t count, unsigned long long* d_mismatches,
                              void* stream) {
  if (!d_mismatches) return fail(PIC_EINVAL, "null mismatch counter");
  if ((uint64_t)first + count > 0x100000000ull) return fail(PIC_EINVAL, "bit range past 2^32");
  if (count == 0) return PIC_OK;
  const unsigned blocks = std::min<unsigned>(8192u, (count + 255u) / 256u);
  hipLaunchKernelGGL(k_check_rounding, dim3(blocks), dim3(256), 0, S(stream), first, count, d_mismatches);
  HIP_TRY(hipGetLastError());
  return PIC_OK;
}

pic_status pic_set_max_grid(pic_run* r, int32_t max_workgroups) {
  if (!r || max_workgroups < 0) return fail(PIC_EINVAL, "null run or negative limit");
  r->max_grid = max_workgroups;
  drop_step_graphs(r);  // the recorded launches follow the limit
  return PIC_OK;
}

pic_status pic_timing_enable(pic_run* r, int32_t period) {
  if (!r) return fail(PIC_EINVAL, "null run");
  if (period < 0) return fail(PIC_EINVAL, "negative timing period");
  if (period) {
    pic_status ps = ev_create(r);
    if (ps) return ps;
  }
  r->timing = period;
  for (auto& k : r->seen) k = 0;
  return PIC_OK;
}

pic_status pic_timing_read(pic_run* r, double ms[3], int64_t launches[3], void* stream) {
  if (!r || !ms || !launches) return fail(PIC_EINVAL, "null argument");
  HIP_TRY(hipStreamSynchronize(S(stream)));
  for (auto& e : r->ev) {
    if (!e.used) continue;
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, e.a, e.b));
    r->ms[e.kind] += t;
    e.used = false;
  }
  for (int k = 0; k < 3; ++k) {
    ms[k] = r->ms[k];
    launches[k] = r->launches[k];
    r->ms[k] = 0.0;
    r->launches[k] = 0;
  }
  return PIC_OK;
}


pic_status pic_batch_workspace_bytes(int32_t precision, int32_t max_slots, size_t* bytes) {
  if (!bytes || max_slots < 1 || max_slots > kMaxSlots || (precision != PIC_FP32 && precision != PIC_FP64))
    return fail(PIC_EINVAL, "bad batch size or precision");
  *bytes = batch_layout(precision, max_slots, nullptr, nullptr);
  return PIC_OK;
}

pic_status pic_batch_create(int32_t precision, int32_t max_slots, int32_t quantum,
                            int64_t max_particles, int64_t max_cells, void* d_ws, size_t ws_bytes,
                            void* stream, pic_batch** out) {
  if (!out) return fail(PIC_EINVAL, "null output handle");
  *out = nullptr;
  size_t need = 0;
  pic_status ps = pic_batch_workspace_bytes(precision, max_slots, &need);
  if (ps) return ps;
  if (!d_ws || reinterpret_cast<uintptr_t>(d_ws) % 256) return fail(PIC_EINVAL, "bad batch workspace");
  if (ws_bytes < need) return fail(PIC_ENOMEM, "batch workspace too small");
  if (quantum < 1 || max_particles < 0 || max_cells < 0) return fail(PIC_EINVAL, "bad batch limits");
  if (!stream) return fail(PIC_EINVAL, "a batch needs a stream other than the null stream (graph capture)");
  pic_batch* b = new pic_batch();
  b->prec = precision;
  b->max_slots = max_slots;
  b->quantum = quantum;
  b->slot_bytes = slot_bytes_for(precision);
  batch_layout(precision, max_slots, b, static_cast<char*>(d_ws));
  b->cap[0] = (int)(max_particles / kBatchTile) + 2 * max_slots;
  b->cap[1] = (int)((max_cells + 3ll * max_slots) / kFieldChunk) + 2 * max_slots;
  b->cap[2] = (int)(max_particles / kSortTile) + 2 * max_slots;
  b->runs.assign(max_slots, nullptr);
  b->target.assign(max_slots, 0);
  b->gen.assign(max_slots, 0);
  b->gen_snap.assign(max_slots, 0);
  if (hipHostMalloc(reinterpret_cast<void**>(&b->pin_steps), (max_slots + 1) * sizeof(long long)) != hipSuccess ||
      hipEventCreateWithFlags(&b->poll_ev, hipEventDisableTiming) != hipSuccess) {
    if (b->pin_steps) (void)hipHostFree(b->pin_steps);
    delete b;
    return fail(PIC_EHIP, "batch poll buffer or event");
  }
  for (int k = 0; k < 4; ++k) b->nblk[k].assign(max_slots, 0);
  hipStream_t st = S(stream);
  hipError_t e = hipMemsetAsync(d_ws, 0, need - 256, st);
  if (e != hipSuccess) {
    pic_batch_free(b);
    return fail(PIC_EHIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
  }
  for (int s = 0; s < max_slots && !ps; ++s)
    ps = precision == PIC_FP32 ? write_slot<float>(b, s, st) : write_slot<double>(b, s, st);
  if (!ps) ps = write_ranges(b, st);
  if (ps) {
    pic_batch_free(b);
    return ps;
  }
  *out = b;
  return PIC_OK;
}

pic_status pic_batch_admit(pic_batch* b, pic_run* r, int64_t n_steps, void* stream, int32_t* slot) {
  if (!b || !r || !slot || n_steps < 0) return fail(PIC_EINVAL, "null batch, run or slot");
  if (r->batch) return fail(PIC_EINVAL, "run is already in a batch");
  if (r->d.prec != b->prec) return fail(PIC_EINVAL, "run precision differs from the batch");
  if (r->step != 0 || r->pp != 0) return fail(PIC_EINVAL, "only runs at step 0 can join a batch");
  if (r->cfg.sort_interval != b->quantum)
    return fail(PIC_EINVAL, "run sort_interval must equal the batch quantum");
  int free_slot = -1;
  for (int s = 0; s < b->max_slots; ++s)
    if (!b->runs[s]) {
      free_slot = s;
      break;
    }
  if (free_slot < 0) return fail(PIC_EBUSY, "no free batch slot");
  int need[4];
  batch_need(r->n_max[0], r->n_max[1], r->d.nx, need);
  for (int k = 0; k < 3; ++k)
    if (need[k] > b->cap[k]) return fail(PIC_EINVAL, "run exceeds the batch's work capacity");
  if (!batch_room(b, need)) return fail(PIC_EBUSY, "batch work capacity exhausted");
  b->runs[free_slot] = r;
  b->target[free_slot] = n_steps;
  for (int k = 0; k < 4; ++k) b->nblk[k][free_slot] = need[k];
  hipStream_t st = S(stream);
  // batched steps use their own tile size: the push's tile ranges restart
  HIP_TRY(hipMemsetAsync(r->tpred, 0, 2 * sizeof(int), st));
  pic_status ps = b->prec == PIC_FP32 ? write_slot<float>(b, free_slot, st) : write_slot<double>(b, free_slot, st);
  if (!ps) ps = write_ranges(b, st);
  if (ps) {
    b->runs[free_slot] = nullptr;
    for (int k = 0; k < 4; ++k) b->nblk[k][free_slot] = 0;
    return ps;
  }
  r->batch = b;
  ++b->gen[free_slot];
  *slot = free_slot;
  return PIC_OK;
}

pic_status pic_batch_fits(const pic_batch* b, const pic_config* cfg, int32_t* now, int32_t* ever) {
  if (!b || !cfg || !now || !ever) return fail(PIC_EINVAL, "null batch, config or output");
  Derived d;
  pic_status ps = derive(cfg, &d);
  if (ps) return ps;
  if (d.prec != b->prec) return fail(PIC_EINVAL, "run precision differs from the batch");
  if (cfg->sort_interval != b->quantum) return fail(PIC_EINVAL, "run sort_interval must equal the batch quantum");
  int need[4];
  batch_need(d.n_foil, d.n_foil, d.nx, need);
  *ever = 1;
  for (int k = 0; k < 3; ++k)
    if (need[k] > b->cap[k]) *ever = 0;
  bool slot = false;
  for (int s = 0; s < b->max_slots; ++s) slot = slot || !b->runs[s];
  *now = (*ever && slot && batch_room(b, need)) ? 1 : 0;
  return PIC_OK;
}

pic_status pic_batch_step(pic_batch* b, int32_t n_quanta, void* stream) {
  if (!b || n_quanta < 0 || !stream) return fail(PIC_EINVAL, "null batch/stream or negative count");
  hipStream_t st = S(stream);
  if (!b->exec) {
    pic_status ps = b->prec == PIC_FP32 ? capture_batch<float>(b, st) : capture_batch<double>(b, st);
    if (!ps) ps = update_batch_grids(b);
    if (ps) return ps;
  }
  for (int q = 0; q < n_quanta; ++q) HIP_TRY(hipGraphLaunch(b->exec, st));
  return PIC_OK;
}

pic_status pic_batch_poll(pic_batch* b, int64_t* steps, void* stream) {
  if (!b || !steps || !stream) return fail(PIC_EINVAL, "null batch, output or stream");
  hipStream_t st = S(stream);
  const size_t off = b->prec == PIC_FP32 ? offsetof(SlotDev<float>, step) : offsetof(SlotDev<double>, step);
  hipLaunchKernelGGL(k_gather_steps, dim3((b->max_slots + 255) / 256), dim3(256), 0, st, b->tab,
                     b->slot_bytes, off, b->max_slots, b->steps);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(steps, b->steps, b->max_slots * sizeof(long long), hipMemcpyDeviceToHost, st));
  int err = 0;
  HIP_TRY(hipMemcpyAsync(&err, b->err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int s = 0; s < b->max_slots; ++s)
    if (!b->runs[s]) steps[s] = -1;
  if (err) return fail(PIC_EHIP, "a persistent batch launch timed out in a grid barrier; its steps are not valid");
  return PIC_OK;
}

pic_status pic_batch_poll_async(pic_batch* b, void* stream) {
  if (!b || !stream) return fail(PIC_EINVAL, "null batch or stream");
  if (b->poll_pending) return fail(PIC_EINVAL, "a poll of this batch is already queued");
  hipStream_t st = S(stream);
  const size_t off = b->prec == PIC_FP32 ? offsetof(SlotDev<float>, step) : offsetof(SlotDev<double>, step);
  hipLaunchKernelGGL(k_gather_steps, dim3((b->max_slots + 255) / 256), dim3(256), 0, st, b->tab,
                     b->slot_bytes, off, b->max_slots, b->steps);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(b->pin_steps, b->steps, b->max_slots * sizeof(long long), hipMemcpyDeviceToHost, st));
  b->pin_steps[b->max_slots] = 0;
  HIP_TRY(hipMemcpyAsync(b->pin_steps + b->max_slots, b->err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(b->poll_ev, st));
  b->gen_snap = b->gen;
  b->poll_pending = true;
  return PIC_OK;
}

pic_status pic_batch_poll_wait(pic_batch* b, int64_t* steps) {
  if (!b || !steps) return fail(PIC_EINVAL, "null batch or output");
  if (!b->poll_pending) return fail(PIC_EINVAL, "no poll of this batch is queued");
  b->poll_pending = false;
  HIP_TRY(hipEventSynchronize(b->poll_ev));
  for (int s = 0; s < b->max_slots; ++s)
    steps[s] = (b->runs[s] && b->gen[s] == b->gen_snap[s]) ? b->pin_steps[s] : -1;
  int err = 0;
  std::memcpy(&err, b->pin_steps + b->max_slots, sizeof(int));
  if (err) return fail(PIC_EHIP, "a persistent batch launch timed out in a grid barrier; its steps are not valid");
  return PIC_OK;
}

pic_status pic_batch_drain(pic_batch* b, int64_t* quanta, void* stream) {
  if (!b || !stream) return fail(PIC_EINVAL, "null batch or stream");
  std::vector<int64_t> steps(b->max_slots);
  int64_t total = 0;
  // every resident run advances in the same quanta, so one round of
  // replays covers the longest remainder; the second poll confirms it
  for (int round = 0; round < 2; ++round) {
    pic_status ps = pic_batch_poll(b, steps.data(), stream);
    if (ps) return ps;
    long long left = 0;
    for (int s = 0; s < b->max_slots; ++s)
      if (b->runs[s]) left = std::max(left, b->target[s] - (long long)steps[s]);
    if (left <= 0) {
      if (quanta) *quanta = total;
      return PIC_OK;
    }
    const long long nq = (left + b->quantum - 1) / b->quantum;
    if (nq > INT32_MAX) return fail(PIC_EINVAL, "remaining steps exceed one drain");
    ps = pic_batch_step(b, (int32_t)nq, stream);
    if (ps) return ps;
    total += nq;
  }
  return fail(PIC_EHIP, "batch runs did not reach their step targets");
}

pic_status pic_batch_set_persistent(pic_batch* b, int32_t on) {
  if (!b || on < 0 || on > 2) return fail(PIC_EINVAL, "null batch or mode other than 0 / 1 / 2");
  if (on && b->max_slots > kPersistSlots)
    return fail(PIC_EINVAL, "persistent batch steps serve at most " + std::to_string(kPersistSlots) + " slots");
  const unsigned long long ticks = on == 2 ? 0ull : kBarTicks;
  if ((on != 0) == b->persistent && ticks == b->bar_ticks) return PIC_OK;
  b->persistent = on != 0;
  b->bar_ticks = ticks;
  // captured again, in the new form, by the next pic_batch_step
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->nodes.clear();
  return PIC_OK;
}

pic_status pic_batch_release(pic_batch* b, int32_t slot, void* stream) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->runs[slot]) return fail(PIC_EINVAL, "bad slot");
  hipStream_t st = S(stream);
  HIP_TRY(hipStreamSynchronize(st));
  pic_run* r = b->runs[slot];
  long long step = 0;
  HIP_TRY(hipMemcpy(&step, r->step_dev, sizeof(step), hipMemcpyDeviceToHost));
  r->step = step;
  // sorts ran at the starts of steps K, 2K, ... below `step`
  r->pp = step > 0 ? (int)(((step - 1) / r->cfg.sort_interval) & 1) : 0;
  r->batch = nullptr;
  HIP_TRY(hipMemsetAsync(r->tpred, 0, 2 * sizeof(int), st));  // single-run tiles from here
  b->runs[slot] = nullptr;
  ++b->gen[slot];
  b->target[slot] = 0;
  for (int k = 0; k < 4; ++k) b->nblk[k][slot] = 0;
  pic_status ps = b->prec == PIC_FP32 ? write_slot<float>(b, slot, st) : write_slot<double>(b, slot, st);
  if (!ps) ps = write_ranges(b, st);
  return ps;
}

void pic_batch_free(pic_batch* b) {
  if (!b) return;
  for (int s = 0; s < b->max_slots; ++s)
    if (b->runs[s]) b->runs[s]->batch = nullptr;
  if (b->poll_ev) {
    if (b->poll_pending) (void)hipEventSynchronize(b->poll_ev);  // the copy into pin_steps ends first
    (void)hipEventDestroy(b->poll_ev);
  }
  if (b->pin_steps) (void)hipHostFree(b->pin_steps);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
}

}  // extern "C"

// The 2D3V entry points share this translation unit and its helpers.
#include "pic2d_host.inc"
