// Host side of the C ABI declared in include/pic.h: workspace carving,
// validation, kernel launches, state I/O and per-kernel event timing.
#include "pic.h"
#include "kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace pic;

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
  d->cap = std::max<long long>(d->n_foil, c->capacity);
  // kernels address particle arrays with 32-bit byte offsets
  const long long elem = c->precision == PIC_FP32 ? 4 : 8;
  if (d->cap < 0 || d->cap * elem > (1ll << 32) - (long long)kTile * elem)
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
  double* budget;       // [4]
  int* cnt[2];
  int* cursor[2];
  long long* rho;
  double* part;
  long long* ipart;
  DiagOutDev* dout;
  unsigned long long* hist;
  int tiles_max;
  // timing
  bool timing = false;
  std::vector<TimingRec> ev;
  size_t ev_next = 0;
  double ms[3] = {0, 0, 0};
  long long launches[3] = {0, 0, 0};
};

namespace {

int tiles_for(long long n) { return (int)((n + kTile - 1) / kTile); }

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
  r->tiles_max = 2 * tiles_for(d.cap);
  r->acc = cv.take<double>(4 * (size_t)std::max(r->tiles_max, 1));
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

pic_status ev_begin(pic_run* r, int kind, hipStream_t st, size_t* slot) {
  if (!r->timing) return PIC_OK;
  if (r->ev.empty()) {
    r->ev.resize(512);
    for (auto& e : r->ev) {
      HIP_TRY(hipEventCreate(&e.a));
      HIP_TRY(hipEventCreate(&e.b));
      e.used = false;
    }
  }
  TimingRec& e = r->ev[r->ev_next];
  if (e.used) {  // ring full: fold the oldest record in
    HIP_TRY(hipEventSynchronize(e.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e.a, e.b));
    r->ms[e.kind] += ms;
    e.used = false;
  }
  e.kind = kind;
  HIP_TRY(hipEventRecord(e.a, st));
  *slot = r->ev_next;
  r->ev_next = (r->ev_next + 1) % r->ev.size();
  return PIC_OK;
}

pic_status ev_end(pic_run* r, hipStream_t st, size_t slot) {
  if (!r->timing) return PIC_OK;
  TimingRec& e = r->ev[slot];
  HIP_TRY(hipEventRecord(e.b, st));
  e.used = true;
  r->launches[e.kind] += 1;
  return PIC_OK;
}

template <typename R>
pic_status launch_push(pic_run* r, hipStream_t st) {
  const Derived& d = r->d;
  const int t0 = tiles_for(r->n_max[0]), t1 = tiles_for(r->n_max[1]);
  if (t0 + t1 == 0) return PIC_OK;
  PushArgs<R> a{};
  for (int s = 0; s < 2; ++s) a.sp[s] = dev<R>(r->sp[s][r->pp]);
  a.count = r->count + 2 * r->pp;
  a.tiles0 = t0;
  a.f = fdev<R>(r, (int)(r->step & 1));
  for (int k = 0; k < 3; ++k) a.J[k] = r->J[r->step & 1][k];
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
  a.comp = (r->cfg.rr && r->cfg.rr_compensated && r->cfg.precision == PIC_FP32) ? 1 : 0;
  a.sw = (R)(256.0 / d.w_ref);
  for (int s = 0; s < 2; ++s)  // the kernel's own rounding of a particle of weight w_ref
    a.qw_ref[s] = a.Z[s] * (int)std::rint((R)d.w_ref * a.sw);
  size_t slot = 0;
  pic_status ps = ev_begin(r, 0, st, &slot);
  if (ps) return ps;
  hipLaunchKernelGGL(k_push<R>, dim3(t0 + t1), dim3(kThreads), 0, st, a);
  HIP_TRY(hipGetLastError());
  return ev_end(r, st, slot);
}

template <typename R>
pic_status launch_field(pic_run* r, hipStream_t st) {
  const Derived& d = r->d;
  const int p = (int)(r->step & 1);
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
  const int blocks = (d.nx + 3 + kFieldChunk - 1) / kFieldChunk;
  size_t slot = 0;
  pic_status ps = ev_begin(r, 1, st, &slot);
  if (ps) return ps;
  hipLaunchKernelGGL(k_field<R>, dim3(blocks), dim3(kFieldChunk), 0, st, f);
  HIP_TRY(hipGetLastError());
  ps = ev_end(r, st, slot);
  if (ps) return ps;
  r->step += 1;
  return PIC_OK;
}

template <typename R>
pic_status launch_sort(pic_run* r, hipStream_t st) {
  const Derived& d = r->d;
  SortArgs<R> p{};
  for (int s = 0; s < 2; ++s) {
    p.src[s] = dev<R>(r->sp[s][r->pp]);
    p.dst[s] = dev<R>(r->sp[s][r->pp ^ 1]);
    p.cnt[s] = r->cnt[s];
    p.cursor[s] = r->cursor[s];
  }
  p.count = r->count + 2 * r->pp;
  p.nx = d.nx;
  p.comp = (r->cfg.rr && r->cfg.rr_compensated && r->cfg.precision == PIC_FP32) ? 1 : 0;
  auto blocks = [](long long n) {
    return (int)std::max<long long>(1, (n + kSortTile - 1) / kSortTile);
  };
  p.blocks0 = blocks(r->n_max[0]);
  const int grid = p.blocks0 + blocks(r->n_max[1]);
  size_t slot = 0;
  pic_status ps = ev_begin(r, 2, st, &slot);
  if (ps) return ps;
  hipLaunchKernelGGL(k_sort_hist<R>, dim3(grid), dim3(kSortThreads), 0, st, p);
  hipLaunchKernelGGL(k_sort_scan, dim3(2), dim3(1024), 0, st, r->cnt[0], r->cnt[1], r->cursor[0],
                     r->cursor[1], r->count + 2 * (r->pp ^ 1), d.nx);
  hipLaunchKernelGGL(k_sort_scatter<R>, dim3(grid), dim3(kSortThreads), 0, st, p);
  HIP_TRY(hipGetLastError());
  ps = ev_end(r, st, slot);
  if (ps) return ps;
  r->pp ^= 1;
  return PIC_OK;
}

template <typename R>
pic_status do_steps(pic_run* r, int64_t n, hipStream_t st) {
  for (int64_t k = 0; k < n; ++k) {
    if (r->step > 0 && r->step % r->cfg.sort_interval == 0) {
      pic_status ps = launch_sort<R>(r, st);
      if (ps) return ps;
    }
    pic_status ps = launch_push<R>(r, st);
    if (ps) return ps;
    ps = launch_field<R>(r, st);
    if (ps) return ps;
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
  if (step_dev != r->step)
    return fail(PIC_EHIP, "device step counter disagrees with the host (lost launch?)");
  if (out->nonfinite) return fail(PIC_ENONFINITE, "a particle momentum became non-finite");
  return PIC_OK;
}

size_t rsz(const pic_run* r) { return r->d.rsize; }

}  // namespace

extern "C" {

const char* pic_last_error(void) { return g_err.c_str(); }

pic_status pic_workspace_bytes(const pic_config* cfg, size_t* bytes) {
  if (!bytes) return fail(PIC_EINVAL, "null bytes pointer");
  pic_run tmp;
  tmp.cfg = *cfg;
  pic_status st = derive(cfg, &tmp.d);
  if (st) return st;
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
  return r->d.prec == PIC_FP32 ? do_steps<float>(r, n, S(stream)) : do_steps<double>(r, n, S(stream));
}

pic_status pic_push_deposit(pic_run* r, void* stream) {
  if (!r) return fail(PIC_EINVAL, "null run");
  return r->d.prec == PIC_FP32 ? launch_push<float>(r, S(stream)) : launch_push<double>(r, S(stream));
}

pic_status pic_field_advance(pic_run* r, void* stream) {
  if (!r) return fail(PIC_EINVAL, "null run");
  return r->d.prec == PIC_FP32 ? launch_field<float>(r, S(stream)) : launch_field<double>(r, S(stream));
}

pic_status pic_sort(pic_run* r, void* stream) {
  if (!r) return fail(PIC_EINVAL, "null run");
  return r->d.prec == PIC_FP32 ? launch_sort<float>(r, S(stream)) : launch_sort<double>(r, S(stream));
}

pic_status pic_diag(pic_run* r, pic_diag_out* out, void* stream) {
  if (!r || !out) return fail(PIC_EINVAL, "null run or output");
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
  o->tile = kTile;
  o->lds_slots = kLdsSlots;
  return PIC_OK;
}

void pic_free(pic_run* r) {
  if (!r) return;
  for (auto& e : r->ev) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  delete r;
}

pic_status pic_get_state(pic_run* r, pic_state* st, void* stream) {
  if (!r || !st) return fail(PIC_EINVAL, "null run or state");
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
  return PIC_OK;
}

pic_status pic_set_state(pic_run* r, const pic_state* st, void* stream) {
  if (!r || !st) return fail(PIC_EINVAL, "null run or state");
  hipStream_t s = S(stream);
  const Derived& d = r->d;
  const size_t rs = rsz(r);
  HIP_TRY(hipStreamSynchronize(s));
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
  HIP_TRY(hipDeviceSynchronize());
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

pic_status pic_timing_enable(pic_run* r, int32_t enable) {
  if (!r) return fail(PIC_EINVAL, "null run");
  r->timing = enable != 0;
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

}  // extern "C"
