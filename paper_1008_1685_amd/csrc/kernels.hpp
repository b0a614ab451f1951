// Device code of the 1D3V PIC hot path with radiation reaction (gfx950).
//
// Kernels (one HIP launch each):
//   k_push      gather -> Boris -> RR (electrons) -> move -> integer deposit,
//               one thread per particle over cell-sorted SoA tiles; current
//               accumulated in lane-private LDS copies of a window of nodes,
//               then one global 64-bit atomic per node and work-group.
//   k_field     1D Yee advance (two B half steps around the E step), laser
//               injection and absorption at the ends, Ex as the integral of
//               the charge flux; one thread per node, halo recomputed.
//   k_sort_*    counting sort of particles by cell (histogram, scan, scatter).
//   k_diag_*    FP64 energy budget and exact integer Gauss check.
//   k_init, k_spectrum: quiet start and ion energy histogram.
//
// Templated on the storage type R (float: precision form, double: plain
// form).  Everything that decides an integer (cell index, fixed-point
// current) is computed with one IEEE rounding per operation and no fused
// multiply-add, in the order fixed by the deposition contract.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <limits.h>

namespace pic {

constexpr int kDead = INT_MIN;        // cell index of a removed particle
constexpr int kThreads = 256;         // push work-group
constexpr int kPPT = 8;               // particles per thread per tile
constexpr int kTile = kThreads * kPPT;
constexpr int kNW = 16;               // LDS deposit window (storage indices)
constexpr int kLanes = 64;            // wavefront width; one LDS copy per lane
constexpr int kFieldChunk = 256;      // nodes per field work-group
constexpr int kTwo24 = 1 << 24;

template <typename R>
struct SpeciesDev {
  int* cell;
  R* off;
  R* ux;
  R* uy;
  R* uz;
  R* w;
  float* rx;  // compensated RR residuals (fp32 electrons), else null
  float* ry;
  float* rz;
};

template <typename R>
struct FieldsDev {
  R* Ex;  // half-nodes 0..n+1
  R* Ey;  // nodes 0..n
  R* Ez;
  R* By;  // half-nodes
  R* Bz;
};

template <typename R>
struct PushArgs {
  SpeciesDev<R> sp[2];
  const long long* count;        // [2] particles per species as of the last sort
  int tiles0;                    // work-groups of species 0
  FieldsDev<R> f;                // E^n, B^n
  unsigned long long* J[3];      // Jx (half-nodes), Jy, Jz (nodes, index node+1)
  double* acc;                   // [tile][4] cumulative: E_rad, E_esc_e, E_esc_i, n_stiff
  int* flags;                    // [0]: non-finite seen
  int nx;
  R cfl;                         // dt / dx
  R dt;
  R eps;                         // RR strength (4 pi / 3) r_e / lambda
  R qh[2];                       // q/m dt / 2 per species
  int Z[2];                      // charge per species
  double mass[2];
  int rr0;                       // RR on species 0 (electrons)
  int comp;                      // compensated RR accumulation (fp32 only)
  R sw;                          // 256 / w_ref (charge-weight scale)
};

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

__device__ __forceinline__ long long wave_sum(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// Position update of the deposition contract: gamma from the stored
// momentum in the order ((1 + ux^2) + uy^2) + uz^2, correctly rounded square
// root and division, displacement vx*cfl, offset renormalised to [0, 1).
template <typename R>
__device__ __forceinline__ void contract_move(R ux, R uy, R uz, R o, R cfl, R& g,
                                              R& vy, R& vz, R& o1, R& s) {
#pragma clang fp contract(off)
  g = sqrt(((R(1) + ux * ux) + uy * uy) + uz * uz);
  const R ig = R(1) / g;
  const R vx = ux * ig;
  vy = uy * ig;
  vz = uz * ig;
  const R d = vx * cfl;
  s = o + d;
  R fl = floor(s);
  o1 = s - fl;
  if (o1 >= R(1)) {
    o1 = R(0);
    fl += R(1);
  }
  s = fl;  // integer cell shift
}

// Knuth's TwoSum: a + b = s + e exactly.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

struct DepositCtx {
  unsigned long long* lds;  // [3][kNW][kLanes]
  unsigned long long* J[3];
  int wlo;                  // storage index of window slot 0
  int lane;
  int jmin, jmax;           // window slots touched by this thread
};

// Integer current of one move (cell c, offset o) -> (c1, o1); see the
// deposition contract in the library header notes.
template <typename R>
__device__ __forceinline__ void deposit(DepositCtx& d, int c, R o, int c1, R o1,
                                        R vy, R vz, int qw) {
  const int q0 = (int)(o * R(kTwo24));
  const int q1 = (int)(o1 * R(kTwo24));
  const int base = min(c, c1);
  const int d0 = c - base, d1 = c1 - base;
  const int wo0 = d0 ? 0 : kTwo24 - q0;
  const int wo1 = d0 ? kTwo24 - q0 : q0;
  const int wo2 = d0 ? q0 : 0;
  const int wn0 = d1 ? 0 : kTwo24 - q1;
  const int wn1 = d1 ? kTwo24 - q1 : q1;
  const int wn2 = d1 ? q1 : 0;
  const int F0 = wo0 - wn0;
  const int F1 = F0 + wo1 - wn1;
  const long long vy24 = (long long)rint(vy * R(kTwo24));
  const long long vz24 = (long long)rint(vz * R(kTwo24));
  const long long jx0 = (long long)qw * F0;
  const long long jy0 = (long long)qw * ((vy24 * (wo0 + wn0)) >> 25);
  const long long jy1 = (long long)qw * ((vy24 * (wo1 + wn1)) >> 25);
  const long long jz0 = (long long)qw * ((vz24 * (wo0 + wn0)) >> 25);
  const long long jz1 = (long long)qw * ((vz24 * (wo1 + wn1)) >> 25);
  const bool moved = (c1 != c);
  const int j0 = base + 1;  // Jx half-node base+1/2 and Jy node base share index base+1
  const int r = j0 - d.wlo;
  if (r >= 0 && r + 2 < kNW) {
    unsigned long long* L = d.lds + d.lane;
    atomicAdd(L + ((0 * kNW + r) << 6), (unsigned long long)jx0);
    atomicAdd(L + ((1 * kNW + r) << 6), (unsigned long long)jy0);
    atomicAdd(L + ((1 * kNW + r + 1) << 6), (unsigned long long)jy1);
    atomicAdd(L + ((2 * kNW + r) << 6), (unsigned long long)jz0);
    atomicAdd(L + ((2 * kNW + r + 1) << 6), (unsigned long long)jz1);
    d.jmin = min(d.jmin, r);
    d.jmax = max(d.jmax, r + 1);
    if (moved) {
      const long long jx1 = (long long)qw * F1;
      const long long jy2 = (long long)qw * ((vy24 * (wo2 + wn2)) >> 25);
      const long long jz2 = (long long)qw * ((vz24 * (wo2 + wn2)) >> 25);
      atomicAdd(L + ((0 * kNW + r + 1) << 6), (unsigned long long)jx1);
      atomicAdd(L + ((1 * kNW + r + 2) << 6), (unsigned long long)jy2);
      atomicAdd(L + ((2 * kNW + r + 2) << 6), (unsigned long long)jz2);
      d.jmax = max(d.jmax, r + 2);
    }
  } else {
    atomicAdd(d.J[0] + j0, (unsigned long long)jx0);
    atomicAdd(d.J[1] + j0, (unsigned long long)jy0);
    atomicAdd(d.J[1] + j0 + 1, (unsigned long long)jy1);
    atomicAdd(d.J[2] + j0, (unsigned long long)jz0);
    atomicAdd(d.J[2] + j0 + 1, (unsigned long long)jz1);
    if (moved) {
      const long long jx1 = (long long)qw * F1;
      const long long jy2 = (long long)qw * ((vy24 * (wo2 + wn2)) >> 25);
      const long long jz2 = (long long)qw * ((vz24 * (wo2 + wn2)) >> 25);
      atomicAdd(d.J[0] + j0 + 1, (unsigned long long)jx1);
      atomicAdd(d.J[1] + j0 + 2, (unsigned long long)jy2);
      atomicAdd(d.J[2] + j0 + 2, (unsigned long long)jz2);
    }
  }
}

struct PushAcc {
  double rad, esc, stiff;
};

// One particle: gather, Boris, RR, move, deposit, store.
template <typename R, bool RR, bool COMP>
__device__ __forceinline__ void push_particle(const PushArgs<R>& a, const SpeciesDev<R>& sp,
                                              int s, int i, DepositCtx& dc, PushAcc& acc) {
  const int c = sp.cell[i];
  if (c == kDead) return;
  const R o = sp.off[i];
  const R ux = sp.ux[i], uy = sp.uy[i], uz = sp.uz[i];
  const R w = sp.w[i];
  float rx = 0.f, ry = 0.f, rz = 0.f;
  if (COMP) {
    rx = sp.rx[i];
    ry = sp.ry[i];
    rz = sp.rz[i];
  }

  // ---- gather E^n, B^n (linear weights; E_y,E_z on nodes, the rest on half-nodes)
  const R on = R(1) - o;
  const R ey = on * a.f.Ey[c] + o * a.f.Ey[c + 1];
  const R ez = on * a.f.Ez[c] + o * a.f.Ez[c + 1];
  const R sx = o + R(0.5);
  const int hb = sx >= R(1);
  const R fh = hb ? sx - R(1) : sx;
  const int h = c + hb;
  const R fn = R(1) - fh;
  const R ex = fn * a.f.Ex[h] + fh * a.f.Ex[h + 1];
  const R by = fn * a.f.By[h] + fh * a.f.By[h + 1];
  const R bz = fn * a.f.Bz[h] + fh * a.f.Bz[h + 1];

  // ---- Boris (B_x = 0 in 1D)
  const R qh = a.qh[s];
  const R hx = qh * ex, hy = qh * ey, hz = qh * ez;
  const R mx = ux + hx, my = uy + hy, mz = uz + hz;
  const R igm = rsq(R(1) + mx * mx + my * my + mz * mz);
  const R ty = qh * by * igm, tz = qh * bz * igm;
  const R sf = R(2) / (R(1) + ty * ty + tz * tz);
  const R px = mx + (my * tz - mz * ty);
  const R py = my - mx * tz;
  const R pz = mz + mx * ty;
  const R sy = sf * ty, sz = sf * tz;
  const R Lx = mx + (py * sz - pz * sy) + hx;
  const R Ly = my - px * sz + hy;
  const R Lz = mz + px * sy + hz;

  R nx = Lx, ny = Ly, nz = Lz;
  R gL = R(0), ddx = R(0), ddy = R(0), ddz = R(0);
  if (RR) {
    // mid-step momentum (u_L + u^{n-1/2}) / 2 and its velocity
    const R qx = R(0.5) * (Lx + ux), qy = R(0.5) * (Ly + uy), qz = R(0.5) * (Lz + uz);
    const R g2 = R(1) + qx * qx + qy * qy + qz * qz;
    const R ig = rsq(g2);
    const R vx = qx * ig, vy = qy * ig, vz = qz * ig;
    // F = E + v x B = -f_L
    const R Fx = ex + (vy * bz - vz * by);
    const R Fy = ey - vx * bz;
    const R Fz = ez + vx * by;
    const R vE = vx * ex + vy * ey + vz * ez;
    R br = Fx * Fx + Fy * Fy + Fz * Fz - vE * vE;
    br = br > R(0) ? br : R(0);
    const R g2b = g2 * br;
    const R k = a.eps * a.dt;
    // dt f_R = dt eps [F x B + (v.E) E - gamma^2 (F^2 - (v.E)^2) v]
    ddx = k * ((Fy * bz - Fz * by) + vE * ex - g2b * vx);
    ddy = k * (vE * ey - Fx * bz - g2b * vy);
    ddz = k * (Fx * by + vE * ez - g2b * vz);
    if (ddx * ddx + ddy * ddy + ddz * ddz > R(0.01) * (Lx * Lx + Ly * Ly + Lz * Lz)) acc.stiff += 1.0;
    if (COMP) {
      // increment plus the residual carried from earlier steps, added by TwoSum;
      // the new rounding residual is carried to the next step
      const float dpx = (float)ddx + rx, dpy = (float)ddy + ry, dpz = (float)ddz + rz;
      float sxx, syy, szz;
      two_sum((float)Lx, dpx, sxx, rx);
      two_sum((float)Ly, dpy, syy, ry);
      two_sum((float)Lz, dpz, szz, rz);
      ddx = dpx;
      ddy = dpy;
      ddz = dpz;
      nx = sxx;
      ny = syy;
      nz = szz;
    } else {
      nx = Lx + ddx;
      ny = Ly + ddy;
      nz = Lz + ddz;
    }
    gL = sqrt(R(1) + Lx * Lx + Ly * Ly + Lz * Lz);
  }

  // ---- move (contract arithmetic)
  R g, vy, vz, o1, shift;
  contract_move<R>(nx, ny, nz, o, a.cfl, g, vy, vz, o1, shift);
  if (!(fabs(shift) < R(4)) || !(g < R(1e30))) {  // NaN/Inf momentum: drop it, raise the flag
    sp.cell[i] = kDead;
    atomicOr(a.flags, 1);
    return;
  }
  const int c1 = c + (int)shift;
  const int qw = a.Z[s] * (int)rint(w * a.sw);
  deposit<R>(dc, c, o, c1, o1, vy, vz, qw);

  if (RR) {
    // gamma_L - gamma_new = -(d . (2 u_L + d)) / (gamma_L + gamma_new)
    const R num = ddx * (R(2) * Lx + ddx) + ddy * (R(2) * Ly + ddy) + ddz * (R(2) * Lz + ddz);
    acc.rad += -(double)w * (double)num / ((double)gL + (double)g);
  }
  if (c1 < 0 || c1 >= a.nx) {
    sp.cell[i] = kDead;
    acc.esc += (double)w * a.mass[s] * ((double)g - 1.0);
  } else {
    sp.cell[i] = c1;
    sp.off[i] = o1;
  }
  sp.ux[i] = nx;
  sp.uy[i] = ny;
  sp.uz[i] = nz;
  if (COMP) {
    sp.rx[i] = rx;
    sp.ry[i] = ry;
    sp.rz[i] = rz;
  }
}

template <typename R, bool RR, bool COMP>
__device__ __forceinline__ void push_tile(const PushArgs<R>& a, int s, int tile, int n, int base,
                                          unsigned long long* lds) {
  __shared__ int s_lo, s_hi;
  __shared__ double s_red[3][kThreads / kLanes];
  const SpeciesDev<R> sp = a.sp[s];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

  // window centred on the cell of the tile's middle particle
  const int mid = min(base + kTile / 2, n - 1);
  const int anchor = sp.cell[mid];
  DepositCtx dc;
  dc.lds = lds;
  dc.J[0] = a.J[0];
  dc.J[1] = a.J[1];
  dc.J[2] = a.J[2];
  dc.wlo = anchor == kDead ? INT_MIN / 2 : anchor + 2 - kNW / 2;
  dc.lane = lane;
  dc.jmin = INT_MAX;
  dc.jmax = INT_MIN;

  {
    ulonglong2* z = reinterpret_cast<ulonglong2*>(lds);
    for (int e = tid; e < 3 * kNW * kLanes / 2; e += kThreads) z[e] = make_ulonglong2(0, 0);
  }
  if (tid == 0) {
    s_lo = INT_MAX;
    s_hi = INT_MIN;
  }
  __syncthreads();

  PushAcc acc{0.0, 0.0, 0.0};
#pragma unroll 2
  for (int k = 0; k < kPPT; ++k) {
    const int i = base + k * kThreads + tid;
    if (i < n) push_particle<R, RR, COMP>(a, sp, s, i, dc, acc);
  }

  // used window range of the work-group
  const int lo = wave_min(dc.jmin), hi = wave_max(dc.jmax);
  if (lane == 0) {
    atomicMin(&s_lo, lo);
    atomicMax(&s_hi, hi);
  }
  const double r0 = wave_sum(acc.rad), r1 = wave_sum(acc.esc), r2 = wave_sum(acc.stiff);
  if (lane == 0) {
    s_red[0][wid] = r0;
    s_red[1][wid] = r1;
    s_red[2][wid] = r2;
  }
  __syncthreads();

  // one global atomic per touched window node and component
  const int wlo = s_lo, whi = s_hi;
  if (wlo <= whi) {
    const int ns = whi - wlo + 1;
    for (int e = wid; e < 3 * ns; e += kThreads / kLanes) {
      const int comp = e / ns, r = wlo + e % ns;
      const long long v = wave_sum((long long)lds[((comp * kNW + r) << 6) + lane]);
      if (lane == 0 && v != 0) atomicAdd(a.J[comp] + dc.wlo + r, (unsigned long long)v);
    }
  }
  if (tid == 0) {
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int w = 0; w < kThreads / kLanes; ++w) {
      t0 += s_red[0][w];
      t1 += s_red[1][w];
      t2 += s_red[2][w];
    }
    double* A = a.acc + 4 * (size_t)tile;
    A[0] += t0;
    A[1 + s] += t1;
    A[3] += t2;
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_push(PushArgs<R> a) {
  __shared__ unsigned long long lds[3 * kNW * kLanes];
  const int tile = blockIdx.x;
  const int s = tile < a.tiles0 ? 0 : 1;
  const int tl = s ? tile - a.tiles0 : tile;
  const int n = (int)a.count[s];
  const int base = tl * kTile;
  if (base >= n) return;
  if (s == 0 && a.rr0) {
    if (a.comp)
      push_tile<R, true, true>(a, s, tile, n, base, lds);
    else
      push_tile<R, true, false>(a, s, tile, n, base, lds);
  } else {
    push_tile<R, false, false>(a, s, tile, n, base, lds);
  }
}

// ---------------------------------------------------------------- fields
template <typename R>
struct FieldArgs {
  FieldsDev<R> in, out;           // E^n, B^n -> E^{n+1}, B^{n+1}
  const long long* J[3];          // current of this step
  unsigned long long* Jnext[3];   // current buffer of the next step, zeroed here
  long long* Ex_int;
  double* budget;                 // [0] E_in, [1] E_out_left, [2] E_out_right
  long long* step;                // device step counter
  int nx;
  R a;                            // dt / dx
  R dt;
  double dtd;
  double sJx, sJy;                // fixed point -> current
  double sEx;                     // fixed point -> Ex
  double ay, az;                  // incident amplitude per component
  double tr, tf, tl;              // rise, flat, fall (1/omega)
};

__device__ __forceinline__ double envelope(double t, double tr, double tf, double tl) {
  if (t <= 0.0) return 0.0;
  if (t < tr) {
    const double s = sin(0.5 * M_PI * t / tr);
    return s * s;
  }
  t -= tr;
  if (t < tf) return 1.0;
  t -= tf;
  if (t < tl) {
    const double c = cos(0.5 * M_PI * t / tl);
    return c * c;
  }
  return 0.0;
}

template <typename R>
__global__ __launch_bounds__(kFieldChunk) void k_field(FieldArgs<R> p) {
  constexpr int CH = kFieldChunk;
  __shared__ R sEy[CH + 3], sEz[CH + 3];      // E^n, nodes i0-2 .. i0+CH
  __shared__ R sBy[CH + 2], sBz[CH + 2];      // B, half-nodes i0-1 .. i0+CH
  __shared__ R sJy[CH + 1], sJz[CH + 1];      // J, nodes i0-1 .. i0+CH-1
  __shared__ R nEy[CH + 1], nEz[CH + 1];      // E^{n+1}, nodes i0-1 .. i0+CH-1
  const int t = threadIdx.x;
  const int i0 = blockIdx.x * CH;
  const int n = p.nx;
  const R a = p.a, ha = R(0.5) * p.a, dt = p.dt;

  for (int k = t; k < CH + 3; k += CH) {
    const int i = i0 - 2 + k;
    const bool ok = i >= 0 && i <= n;
    sEy[k] = ok ? p.in.Ey[i] : R(0);
    sEz[k] = ok ? p.in.Ez[i] : R(0);
  }
  for (int k = t; k < CH + 2; k += CH) {
    const int h = i0 - 1 + k;
    const bool ok = h >= 0 && h <= n + 1;
    sBy[k] = ok ? p.in.By[h] : R(0);
    sBz[k] = ok ? p.in.Bz[h] : R(0);
  }
  for (int k = t; k < CH + 1; k += CH) {
    const int i = i0 - 1 + k;
    const bool ok = i >= 0 && i <= n;
    sJy[k] = ok ? (R)((double)p.J[1][i + 1] * p.sJy) : R(0);
    sJz[k] = ok ? (R)((double)p.J[2][i + 1] * p.sJy) : R(0);
  }
  __syncthreads();

  // B^n -> B^{n+1/2} on interior half-nodes h = 1..n
  for (int k = t; k < CH + 2; k += CH) {
    const int h = i0 - 1 + k;
    if (h >= 1 && h <= n) {
      sBz[k] -= ha * (sEy[k + 1] - sEy[k]);
      sBy[k] += ha * (sEz[k + 1] - sEz[k]);
    }
  }
  __syncthreads();

  // boundary guards at t_{n+1/2} (first-order Silver-Mueller with injection)
  double ey_in = 0.0, ez_in = 0.0;
  if (t == 0 && i0 == 0) {
    const double th = ((double)*p.step + 0.5) * p.dtd;
    const double f = envelope(th, p.tr, p.tf, p.tl);
    ey_in = p.ay * f * sin(th);
    ez_in = p.az * f * cos(th);
    // h = 0 is LDS index 1; node 0 is sEy index 2, Jy node 0 is sJy index 1
    const R d = R(1) + a;
    sBz[1] = (R(4) * (R)ey_in - R(2) * sEy[2] - (R(1) - a) * sBz[2] + dt * sJy[1]) / d;
    sBy[1] = (R(2) * sEz[2] - (R(1) - a) * sBy[2] - dt * sJz[1] - R(4) * (R)ez_in) / d;
  }
  if (t == 0 && n + 1 >= i0 && n + 1 <= i0 + CH) {
    const int k = n + 1 - (i0 - 1);       // LDS index of h = n+1
    const int kn = n - (i0 - 2);          // LDS index of node n in sEy
    const int kj = n - (i0 - 1);          // LDS index of node n in sJy
    const R d = R(1) + a;
    sBz[k] = (R(2) * sEy[kn] - (R(1) - a) * sBz[k - 1] - dt * sJy[kj]) / d;
    sBy[k] = (R(-2) * sEz[kn] - (R(1) - a) * sBy[k - 1] + dt * sJz[kj]) / d;
  }
  __syncthreads();

  // E^n -> E^{n+1} on nodes i0-1 .. i0+CH-1
  for (int k = t; k < CH + 1; k += CH) {
    const int i = i0 - 1 + k;
    if (i >= 0 && i <= n) {
      nEy[k] = sEy[k + 1] - a * (sBz[k + 1] - sBz[k]) - dt * sJy[k];
      nEz[k] = sEz[k + 1] + a * (sBy[k + 1] - sBy[k]) - dt * sJz[k];
    } else {
      nEy[k] = R(0);
      nEz[k] = R(0);
    }
  }
  __syncthreads();

  // boundary bookkeeping at t_{n+1/2}
  if (t == 0 && i0 == 0) {
    const double eyl = 0.5 * ((double)sEy[2] + (double)nEy[1]);
    const double ezl = 0.5 * ((double)sEz[2] + (double)nEz[1]);
    const double bzl = 0.5 * ((double)sBz[1] + (double)sBz[2]);
    const double byl = 0.5 * ((double)sBy[1] + (double)sBy[2]);
    const double L1 = eyl - bzl, L2 = ezl + byl;
    p.budget[0] += p.dtd * (ey_in * ey_in + ez_in * ez_in);
    p.budget[1] += p.dtd * 0.25 * (L1 * L1 + L2 * L2);
    *p.step += 1;
  }
  if (t == 0 && i0 <= n && n < i0 + CH) {
    const int kn = n - (i0 - 2), ke = n - (i0 - 1), kb = n - (i0 - 1);
    const double eyr = 0.5 * ((double)sEy[kn] + (double)nEy[ke]);
    const double ezr = 0.5 * ((double)sEz[kn] + (double)nEz[ke]);
    const double bzr = 0.5 * ((double)sBz[kb] + (double)sBz[kb + 1]);
    const double byr = 0.5 * ((double)sBy[kb] + (double)sBy[kb + 1]);
    const double R1 = eyr + bzr, R2 = ezr - byr;
    p.budget[2] += p.dtd * 0.25 * (R1 * R1 + R2 * R2);
  }

  // own outputs: node i = i0 + t, half-node h = i0 + t
  const int i = i0 + t;
  if (i <= n) {
    p.out.Ey[i] = nEy[t + 1];
    p.out.Ez[i] = nEz[t + 1];
  }
  const int h = i0 + t;
  if (h <= n + 1) {
    R bz, byv;
    if (h >= 1 && h <= n) {  // B^{n+1/2} -> B^{n+1}
      bz = sBz[t + 1] - ha * (nEy[t + 1] - nEy[t]);
      byv = sBy[t + 1] + ha * (nEz[t + 1] - nEz[t]);
    } else {                 // guards keep their t_{n+1/2} value
      bz = sBz[t + 1];
      byv = sBy[t + 1];
    }
    p.out.Bz[h] = bz;
    p.out.By[h] = byv;
    const long long ex = p.Ex_int[h] - p.J[0][h];
    p.Ex_int[h] = ex;
    p.out.Ex[h] = (R)((double)ex * p.sEx);
    p.Jnext[0][h] = 0ull;
  }
  if (i0 + t <= n + 2) {
    p.Jnext[1][i0 + t] = 0ull;
    p.Jnext[2][i0 + t] = 0ull;
  }
}

// ---------------------------------------------------------------- sort
template <typename R>
struct SortArgs {
  SpeciesDev<R> src[2], dst[2];
  const long long* count;  // [2] particles in the source arrays
  int* cnt[2];          // [n] per-cell counts (zero on entry to k_sort_hist)
  int* cursor[2];       // [n] scatter cursors
  int blocks0;          // blocks of species 0 in hist / scatter grids
  int nx;
  int comp;             // carry residuals of species 0
};

constexpr int kSortThreads = 256;

// wave-aggregated atomicAdd(ptr[key], 1) returning each lane's slot
__device__ __forceinline__ int wave_claim(int* ptr, int key, bool valid) {
  const int lane = threadIdx.x & 63;
  unsigned long long active = __ballot(valid);
  int slot = 0;
  while (active) {
    const int leader = __ffsll((long long)active) - 1;
    const int lk = __shfl(key, leader);
    const unsigned long long same = __ballot(valid && key == lk) & active;
    int base = 0;
    if (lane == leader) base = atomicAdd(ptr + lk, __popcll(same));
    base = __shfl(base, leader);
    if ((same >> lane) & 1ull) slot = base + __popcll(same & ((1ull << lane) - 1ull));
    active &= ~same;
  }
  return slot;
}

template <typename R>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(SortArgs<R> p) {
  const int s = blockIdx.x < p.blocks0 ? 0 : 1;
  const int b = s ? blockIdx.x - p.blocks0 : blockIdx.x;
  const int nb = s ? gridDim.x - p.blocks0 : p.blocks0;
  const long long n = p.count[s];
  for (long long i0 = (long long)b * kSortThreads; i0 < n; i0 += (long long)nb * kSortThreads) {
    const long long i = i0 + threadIdx.x;
    const int c = i < n ? p.src[s].cell[i] : kDead;
    wave_claim(p.cnt[s], c, c != kDead);
  }
}

// exclusive scan of the per-cell counts; one work-group per species; the
// alive count goes to new_count (the count slot of the destination arrays)
__global__ __launch_bounds__(1024) void k_sort_scan(int* cnt0, int* cnt1, int* cur0, int* cur1,
                                                    long long* new_count, int nx) {
  __shared__ int part[1024];
  int* cnt = blockIdx.x ? cnt1 : cnt0;
  int* cur = blockIdx.x ? cur1 : cur0;
  const int t = threadIdx.x;
  const int per = (nx + 1023) / 1024;
  const int lo = min(nx, t * per), hi = min(nx, lo + per);
  int sum = 0;
  for (int j = lo; j < hi; ++j) sum += cnt[j];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - sum;
  for (int j = lo; j < hi; ++j) {
    const int c = cnt[j];
    cur[j] = run;
    run += c;
    cnt[j] = 0;
  }
  if (t == 1023) new_count[blockIdx.x] = part[1023];
}

template <typename R>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(SortArgs<R> p) {
  const int s = blockIdx.x < p.blocks0 ? 0 : 1;
  const int b = s ? blockIdx.x - p.blocks0 : blockIdx.x;
  const int nb = s ? gridDim.x - p.blocks0 : p.blocks0;
  const long long n = p.count[s];
  const SpeciesDev<R> src = p.src[s], dst = p.dst[s];
  const bool comp = s == 0 && p.comp;
  for (long long i0 = (long long)b * kSortThreads; i0 < n; i0 += (long long)nb * kSortThreads) {
    const long long i = i0 + threadIdx.x;
    const int c = i < n ? src.cell[i] : kDead;
    const int j = wave_claim(p.cursor[s], c, c != kDead);
    if (c != kDead) {
      dst.cell[j] = c;
      dst.off[j] = src.off[i];
      dst.ux[j] = src.ux[i];
      dst.uy[j] = src.uy[i];
      dst.uz[j] = src.uz[i];
      dst.w[j] = src.w[i];
      if (comp) {
        dst.rx[j] = src.rx[i];
        dst.ry[j] = src.ry[i];
        dst.rz[j] = src.rz[i];
      }
    }
  }
}

// ---------------------------------------------------------------- init
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long seed,
                                                         unsigned long long i) {
  unsigned long long z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename R>
__global__ void k_init(SpeciesDev<R> e, SpeciesDev<R> ion, long long n, int c0, int ppc,
                       unsigned long long seed, double jitter, R w) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = (int)(i % ppc);
  const R U = (R)(splitmix64(seed, (unsigned long long)i) >> 40) * R(1.0 / 16777216.0);
  R o = ((R)k + R(0.5) + (R)jitter * (U - R(0.5))) / (R)ppc;
  if (!(o < R(1))) o = R(0);
  const int c = c0 + (int)(i / ppc);
  SpeciesDev<R> sp[2] = {e, ion};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    sp[s].cell[i] = c;
    sp[s].off[i] = o;
    sp[s].ux[i] = R(0);
    sp[s].uy[i] = R(0);
    sp[s].uz[i] = R(0);
    sp[s].w[i] = w;
    if (sp[s].rx) {
      sp[s].rx[i] = 0.f;
      sp[s].ry[i] = 0.f;
      sp[s].rz[i] = 0.f;
    }
  }
}

// ---------------------------------------------------------------- diagnostics
constexpr int kDiagThreads = 256;
constexpr int kDiagPartBlocks = 512;   // per species, kinetic energy partials
constexpr int kDiagFieldBlocks = 256;

template <typename R>
struct DiagArgs {
  SpeciesDev<R> sp[2];
  const long long* count;
  FieldsDev<R> f;
  const long long* Ex_int;
  long long* rho;        // [n + 3] integer charge on nodes (index node + 1), zeroed by caller
  double* part;          // partials: [2][kDiagPartBlocks] kinetic, [3][kDiagFieldBlocks] fields
  long long* ipart;      // [kDiagFieldBlocks] gauss max, [2][kDiagPartBlocks] alive counts
  int nx;
  double mass[2];
  int Z[2];
  R sw;
  double dx;
};

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  return t;
}

__device__ __forceinline__ long long wave_sum_ll(long long v) { return wave_sum(v); }

template <typename R>
__global__ __launch_bounds__(kDiagThreads) void k_diag_particles(DiagArgs<R> p) {
  __shared__ double sh[kDiagThreads / 64];
  const int s = blockIdx.x < kDiagPartBlocks ? 0 : 1;
  const int b = blockIdx.x - s * kDiagPartBlocks;
  const long long n = p.count[s];
  const SpeciesDev<R> sp = p.sp[s];
  double ke = 0.0;
  long long alive = 0;
  for (long long i0 = (long long)b * kDiagThreads; i0 < n;
       i0 += (long long)kDiagPartBlocks * kDiagThreads) {
    const long long i = i0 + threadIdx.x;
    int c = kDead;
    R o = R(0);
    int qw = 0;
    if (i < n) {
      c = sp.cell[i];
      if (c != kDead) {
        const double ux = sp.ux[i], uy = sp.uy[i], uz = sp.uz[i];
        const double g = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
        ke += (double)sp.w[i] * p.mass[s] * (g - 1.0);
        o = sp.off[i];
        qw = p.Z[s] * (int)rint(sp.w[i] * p.sw);
        alive += 1;
      }
    }
    // integer charge: wave-aggregate equal cells, then one atomic per cell
    const bool valid = c != kDead;
    const int q = valid ? (int)(o * R(kTwo24)) : 0;
    const long long r0 = (long long)qw * (kTwo24 - q), r1 = (long long)qw * q;
    const int lane = threadIdx.x & 63;
    unsigned long long active = __ballot(valid);
    while (active) {
      const int leader = __ffsll((long long)active) - 1;
      const int lc = __shfl(c, leader);
      const bool mine = valid && c == lc && ((active >> lane) & 1ull);
      const long long a0 = wave_sum(mine ? r0 : 0ll);
      const long long a1 = wave_sum(mine ? r1 : 0ll);
      if (lane == leader) {
        atomicAdd((unsigned long long*)p.rho + lc + 1, (unsigned long long)a0);
        atomicAdd((unsigned long long*)p.rho + lc + 2, (unsigned long long)a1);
      }
      active &= ~__ballot(mine);
    }
  }
  const double t = block_sum(ke, sh);
  const long long na = wave_sum((long long)alive);
  __shared__ long long sa[kDiagThreads / 64];
  if ((threadIdx.x & 63) == 0) sa[threadIdx.x >> 6] = na;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tot = 0;
    for (int w = 0; w < kDiagThreads / 64; ++w) tot += sa[w];
    p.part[s * kDiagPartBlocks + b] = t;
    p.ipart[kDiagFieldBlocks + s * kDiagPartBlocks + b] = tot;
  }
}

template <typename R>
__global__ __launch_bounds__(kDiagThreads) void k_diag_fields(DiagArgs<R> p) {
  __shared__ double sh[kDiagThreads / 64];
  __shared__ long long sm[kDiagThreads / 64];
  const int n = p.nx;
  double ux = 0.0, ue = 0.0, ub = 0.0;
  long long gmax = 0;
  for (int i = blockIdx.x * kDiagThreads + threadIdx.x; i <= n;
       i += kDiagFieldBlocks * kDiagThreads) {
    const double wn = (i == 0 || i == n) ? 0.5 : 1.0;
    const double ey = p.f.Ey[i], ez = p.f.Ez[i];
    ue += wn * (ey * ey + ez * ez);
    if (i >= 1) {  // half-node h = i covers cell i-1
      const double ex = p.f.Ex[i], by = p.f.By[i], bz = p.f.Bz[i];
      ux += ex * ex;
      ub += by * by + bz * bz;
    }
    if (i >= 1 && i <= n - 1) {
      long long r = p.Ex_int[i + 1] - p.Ex_int[i] - p.rho[i + 1];
      r = r < 0 ? -r : r;
      gmax = r > gmax ? r : gmax;
    }
  }
  const double t0 = block_sum(ux, sh);
  const double t1 = block_sum(ue, sh);
  const double t2 = block_sum(ub, sh);
  long long g = gmax;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const long long v = __shfl_xor(g, o);
    g = v > g ? v : g;
  }
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = g;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long m = 0;
    for (int w = 0; w < kDiagThreads / 64; ++w) m = sm[w] > m ? sm[w] : m;
    const int base = 2 * kDiagPartBlocks;
    p.part[base + blockIdx.x] = 0.5 * p.dx * t0;
    p.part[base + kDiagFieldBlocks + blockIdx.x] = 0.5 * p.dx * t1;
    p.part[base + 2 * kDiagFieldBlocks + blockIdx.x] = 0.5 * p.dx * t2;
    p.ipart[blockIdx.x] = m;
  }
}

// Final reduction in fixed order into the diagnostics record.
struct DiagOutDev {
  double U_Ex, U_Et, U_B, K_e, K_i, E_rad, E_esc, n_stiff;
  long long gauss_int, alive0, alive1;
};

__global__ void k_diag_final(const double* part, const long long* ipart, const double* acc,
                             int tiles, DiagOutDev* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  DiagOutDev o{};
  for (int b = 0; b < kDiagPartBlocks; ++b) {
    o.K_e += part[b];
    o.K_i += part[kDiagPartBlocks + b];
    o.alive0 += ipart[kDiagFieldBlocks + b];
    o.alive1 += ipart[kDiagFieldBlocks + kDiagPartBlocks + b];
  }
  const int base = 2 * kDiagPartBlocks;
  for (int b = 0; b < kDiagFieldBlocks; ++b) {
    o.U_Ex += part[base + b];
    o.U_Et += part[base + kDiagFieldBlocks + b];
    o.U_B += part[base + 2 * kDiagFieldBlocks + b];
    o.gauss_int = ipart[b] > o.gauss_int ? ipart[b] : o.gauss_int;
  }
  for (int t = 0; t < tiles; ++t) {
    o.E_rad += acc[4 * t];
    o.E_esc += acc[4 * t + 1] + acc[4 * t + 2];
    o.n_stiff += acc[4 * t + 3];
  }
  *out = o;
}

// ---------------------------------------------------------------- spectrum
template <typename R>
__global__ void k_spectrum(SpeciesDev<R> sp, const long long* count, unsigned long long* hist,
                           int bins, double e_max, double mc2, R sw) {
  const long long n = *count;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    if (sp.cell[i] == kDead) continue;
    const double ux = sp.ux[i], uy = sp.uy[i], uz = sp.uz[i];
    const double E = (sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0) * mc2;
    const long long b = (long long)floor(E / e_max * bins);
    if (b >= 0 && b < bins) {
      const int qw = (int)rint(sp.w[i] * sw);
      atomicAdd(hist + b, (unsigned long long)(long long)qw);
    }
  }
}

}  // namespace pic
