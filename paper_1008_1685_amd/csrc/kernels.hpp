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

#ifndef PIC_PUSH_PPT
#define PIC_PUSH_PPT 20
#endif
#ifndef PIC_BATCH_PPT
#define PIC_BATCH_PPT 4
#endif
#ifndef PIC_PUSH_LDS_SLOTS
#define PIC_PUSH_LDS_SLOTS 3072
#endif
#ifndef PIC_PUSH_DEPTH
#define PIC_PUSH_DEPTH 4
#endif
#ifndef PIC_RING_UNROLL
#define PIC_RING_UNROLL 2
#endif

#ifndef PIC_PUSH_MIN_WAVES
#define PIC_PUSH_MIN_WAVES 0
#endif

constexpr int kDead = INT_MIN;        // cell index of a removed particle
constexpr int kThreads = 256;         // push work-group
constexpr int kPPT = PIC_PUSH_PPT;    // particles per thread per tile (single runs)
constexpr int kTile = kThreads * kPPT;
// Batched runs are small and many: a shorter tile lowers the latency of a
// step of one run (the window set-up and flush are paid over fewer pushes).
constexpr int kBatchPPT = PIC_BATCH_PPT;
constexpr int kBatchTile = kThreads * kBatchPPT;
#ifndef PIC_BATCH_DEPTH
#define PIC_BATCH_DEPTH 2
#endif
// The batched push keeps two particles' loads in flight per thread rather
// than the whole tile's: fewer registers, six waves per SIMD instead of five.
constexpr int kBatchDepth = PIC_BATCH_DEPTH;
constexpr int kMinTile = kTile < kBatchTile ? kTile : kBatchTile;
constexpr int kLdsSlots = PIC_PUSH_LDS_SLOTS;  // 64-bit LDS current accumulators per work-group
constexpr int kDepth = PIC_PUSH_DEPTH;        // particles per thread whose loads are in flight
constexpr int kRingUnroll = PIC_RING_UNROLL;  // ring turns per loop iteration (renames, no copies)
constexpr int kLanes = 64;            // wavefront width
#ifndef PIC_STEPS_MIN_WAVES
#define PIC_STEPS_MIN_WAVES 4  // waves per SIMD the persistent batched-step kernel is compiled for
#endif
#ifndef PIC_STEPS_BLOCKS_PER_CU
#define PIC_STEPS_BLOCKS_PER_CU 0  // work-groups per CU of the persistent launch (0: as many as fit)
#endif
#ifndef PIC_FIELD_CHUNK
#define PIC_FIELD_CHUNK 64
#endif
constexpr int kFieldChunk = PIC_FIELD_CHUNK;  // nodes per field work-group
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
  R* oy;      // y offsets on a 2D grid, else null
};

// Grid fields, interleaved so that one particle gathers with four loads:
//   N[i] = (E_y, E_z) at node i = 0..n,
//   H[h] = (E_x, B_y, B_z, 0) at half-node h = 0..n+1 (x = (h - 1/2) dx).
template <typename R>
struct alignas(2 * sizeof(R)) NodeF {
  R ey, ez;
};
template <typename R>
struct alignas(16) HalfF {
  R ex, by, bz, pad;
};

template <typename R>
struct FieldsDev {
  NodeF<R>* N;
  HalfF<R>* H;
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
  int qw_ref[2];                 // charge weight of a particle of weight w_ref
  int ntiles;                    // tiles of both species
  int tile0;                     // first tile of this launch (a step may be split over launches)
  // Cell range of every tile after the previous push (the particles' cells
  // now, as long as no sort or state change came between): with *pred_in
  // set, a tile sizes its current window from it instead of a pass over its
  // cells.  Only a hint: a particle outside the window deposits by global
  // atomics.  The push writes the next ranges and sets *pred_out.
  const int* rng_in;             // [tile][2] min, max
  int* rng_out;
  const int* pred_in;
  int* pred_out;
};

// ---------------------------------------------------------------- helpers
// Approximate (about 1 ulp) reciprocal, reciprocal square root and square
// root for the Boris and RR arithmetic; the contract lines use IEEE ops.
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }

// Element i of an array at a wave-uniform base: a 32-bit byte offset added
// to the 64-bit base lets the compiler use scalar-base addressing instead of
// per-lane 64-bit address arithmetic.  Arrays stay below 4 GiB (capacity
// limits in the host code).
template <typename T>
__device__ __forceinline__ T ld(const T* p, unsigned i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) +
                                     (size_t)(i * (unsigned)sizeof(T)));
}
// The empty asm re-creates the 32-bit offset in the store's own basic block:
// instruction selection works per block and matches the scalar-base form
// only when it sees the zero extension of the offset, which after the
// push's branches it otherwise does not (a 64-bit add per store).
template <typename T>
__device__ __forceinline__ void st(T* p, unsigned i, T v) {
  unsigned o = i * (unsigned)sizeof(T);
  asm volatile("" : "+v"(o));
  *reinterpret_cast<T*>(reinterpret_cast<char*>(p) + (size_t)o) = v;
}

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

// Row-local reductions with DPP lane shifts (rows of 16 lanes).  After the
// steps 1, 2, .., N/2 of an inclusive shift-and-combine scan, the last lane of
// every aligned group of N lanes holds the group's result.  All lanes of the
// wave must be active.  Lanes shifted in from outside the row read `old`.
template <int N>
__device__ __forceinline__ int row_shr(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, 0x110 + N, 0xf, 0xf, false);
}
template <int N>
__device__ __forceinline__ unsigned long long row_shr64(unsigned long long v) {
  const unsigned lo = (unsigned)row_shr<N>(0, (int)(unsigned)v);
  const unsigned hi = (unsigned)row_shr<N>(0, (int)(unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}
// sum over aligned groups of g lanes, g in {1, 2, 4, 8, 16} (wave-uniform)
__device__ __forceinline__ long long group_sum(long long v, int g) {
  if (g >= 2) v += (long long)row_shr64<1>((unsigned long long)v);
  if (g >= 4) v += (long long)row_shr64<2>((unsigned long long)v);
  if (g >= 8) v += (long long)row_shr64<4>((unsigned long long)v);
  if (g >= 16) v += (long long)row_shr64<8>((unsigned long long)v);
  return v;
}
// wave sum in a fixed order: rows by DPP, then the four row sums
__device__ __forceinline__ double wave_sum_dpp(double x) {
  unsigned long long b = __double_as_longlong(x);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    unsigned long long t = 0;
    switch (k) {
      case 0: t = row_shr64<1>(b); break;
      case 1: t = row_shr64<2>(b); break;
      case 2: t = row_shr64<4>(b); break;
      default: t = row_shr64<8>(b); break;
    }
    b = __double_as_longlong(__longlong_as_double(b) + __longlong_as_double(t));
  }
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  double r[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    r[k] = __longlong_as_double(((long long)__builtin_amdgcn_readlane((int)hi, 16 * k + 15) << 32) |
                                (unsigned)__builtin_amdgcn_readlane((int)lo, 16 * k + 15));
  return (r[0] + r[1]) + (r[2] + r[3]);
}
// wave minimum and maximum, wave-uniform results
__device__ __forceinline__ int wave_min_dpp(int v) {
  v = min(v, row_shr<1>(v, v));
  v = min(v, row_shr<2>(v, v));
  v = min(v, row_shr<4>(v, v));
  v = min(v, row_shr<8>(v, v));
  return min(min(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31)),
             min(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63)));
}
__device__ __forceinline__ int wave_max_dpp(int v) {
  v = max(v, row_shr<1>(v, v));
  v = max(v, row_shr<2>(v, v));
  v = max(v, row_shr<4>(v, v));
  v = max(v, row_shr<8>(v, v));
  return max(max(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31)),
             max(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63)));
}

// Correctly rounded square root and reciprocal for arguments >= 1, from the
// hardware estimates (within one ulp) and exact FMA residuals: the root
// picks among s - ulp, s, s + ulp by the signs of x - s' s; the reciprocal
// takes one Newton step r + r (1 - x r).  Compared exhaustively with the
// compiler's correctly rounded sqrtf and 1.0f / x (pic_check_rounding), they
// agree on every float in [1, 2^128) and [1, 2^126) respectively; infinity
// and NaN propagate.
__device__ __forceinline__ float sqrt_rn_ge1(float x) {
  const float s = __builtin_amdgcn_sqrtf(x);
  const float sd = __int_as_float(__float_as_int(s) - 1), su = __int_as_float(__float_as_int(s) + 1);
  const float rd = fmaf(-sd, s, x), ru = fmaf(-su, s, x);
  const float r = rd <= 0.f ? sd : s;
  return ru > 0.f ? su : r;
}
__device__ __forceinline__ float rcp_rn_ge1(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(fmaf(-x, r, 1.0f), r, r);
}
__device__ __forceinline__ double sqrt_rn_ge1(double x) { return sqrt(x); }
__device__ __forceinline__ double rcp_rn_ge1(double x) { return 1.0 / x; }

// Position update of the deposition contract: gamma from the stored
// momentum in the order ((1 + ux^2) + uy^2) + uz^2, correctly rounded square
// root and division, displacement vx*cfl, offset renormalised to [0, 1).
template <typename R>
__device__ __forceinline__ void contract_move(R ux, R uy, R uz, R o, R cfl, R& g,
                                              R& vy, R& vz, R& o1, R& s) {
#pragma clang fp contract(off)
  g = sqrt_rn_ge1(((R(1) + ux * ux) + uy * uy) + uz * uz);
  const R ig = rcp_rn_ge1(g);
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

// Current accumulation of one push work-group: an LDS window of W storage
// indices (starting at wlo) covering every node the tile's particles can
// touch, with R = 2^k private copies per slot (lane & (R - 1) picks the
// copy), so lanes of a wave that hit the same node add to different words.
// Tiles whose window does not fit use global atomics instead.
struct DepositCtx {
  // current / qw_ref of particles with qw == qw_ref: slot (comp, cell) of
  // copy k at lds[(comp * W + cell) * P + k], P = R + 1 (R > 1) or 1; the
  // odd stride spreads one copy of neighbouring slots over distinct banks
  unsigned long long* lds;
  unsigned long long* J[3];
  int wlo;
  int W;
  int P;
  int copy;
  int qw_ref;
  bool use_lds;
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
  const int vy24 = (int)rint(vy * R(kTwo24));  // |v| < 1: |vy24| <= 2^24
  const int vz24 = (int)rint(vz * R(kTwo24));
  // unweighted Jy, Jz terms: floor(v24 (Wo + Wn) / 2^25), |term| <= 2^24
  const int ty0 = (int)(((long long)vy24 * (wo0 + wn0)) >> 25);
  const int ty1 = (int)(((long long)vy24 * (wo1 + wn1)) >> 25);
  const int ty2 = (int)(((long long)vy24 * (wo2 + wn2)) >> 25);
  const int tz0 = (int)(((long long)vz24 * (wo0 + wn0)) >> 25);
  const int tz1 = (int)(((long long)vz24 * (wo1 + wn1)) >> 25);
  const int tz2 = (int)(((long long)vz24 * (wo2 + wn2)) >> 25);
  const bool moved = (c1 != c);
  const int j0 = base + 1;  // Jx half-node base+1/2 and Jy node base share index base+1
  const int r = j0 - d.wlo;  // 0 <= r <= W - 3 when the particle's cell is in the window
  if (d.use_lds && qw == d.qw_ref && (unsigned)r <= (unsigned)(d.W - 3)) {
    // LDS holds sums of unweighted terms; the flush multiplies by qw_ref
    // slot (comp, r + k) of this lane's copy: x0 + comp * cs + k * ss
    const int ss = d.P, cs = d.W * d.P;
    unsigned long long* x0 = d.lds + d.copy + r * d.P;
    unsigned long long* y0 = x0 + cs;
    unsigned long long* z0 = y0 + cs;
    atomicAdd(x0, (unsigned long long)(long long)F0);
    atomicAdd(y0, (unsigned long long)(long long)ty0);
    atomicAdd(y0 + ss, (unsigned long long)(long long)ty1);
    atomicAdd(z0, (unsigned long long)(long long)tz0);
    atomicAdd(z0 + ss, (unsigned long long)(long long)tz1);
    if (moved) {
      atomicAdd(x0 + ss, (unsigned long long)(long long)F1);
      atomicAdd(y0 + 2 * ss, (unsigned long long)(long long)ty2);
      atomicAdd(z0 + 2 * ss, (unsigned long long)(long long)tz2);
    }
  } else {
    // keep the 64-bit products of this rare path out of the common one
    int F1m = F1, ty2m = ty2, tz2m = tz2;
    int t[5] = {F0, ty0, ty1, tz0, tz1};
    asm volatile("" : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]), "+v"(F1m), "+v"(ty2m),
                 "+v"(tz2m));
    const long long q = qw;
    atomicAdd(d.J[0] + j0, (unsigned long long)(q * t[0]));
    atomicAdd(d.J[1] + j0, (unsigned long long)(q * t[1]));
    atomicAdd(d.J[1] + j0 + 1, (unsigned long long)(q * t[2]));
    atomicAdd(d.J[2] + j0, (unsigned long long)(q * t[3]));
    atomicAdd(d.J[2] + j0 + 1, (unsigned long long)(q * t[4]));
    if (moved) {
      atomicAdd(d.J[0] + j0 + 1, (unsigned long long)(q * F1m));
      atomicAdd(d.J[1] + j0 + 2, (unsigned long long)(q * ty2m));
      atomicAdd(d.J[2] + j0 + 2, (unsigned long long)(q * tz2m));
    }
  }
}

// per-thread partial sums (a thread pushes the PPT particles of its tile; FP64 from the
// work-group sum on)
struct PushAcc {
  float rad, esc, stiff;
  int cmin1, cmax1;  // range of the new cells of the thread's particles
};

// Stored state of one particle (besides its cell).
template <typename R>
struct PData {
  int c;
  R o, ux, uy, uz, w;
  float rx, ry, rz;
};

// Partial derivatives of the fields at a particle, for the derivative term of
// Eq. (3dLL): d/dt and d/dx of E_x, E_y, E_z, B_y, B_z (B_x = 0 in 1D).
template <typename R>
struct FieldRates {
  R etx, ety, etz, bty, btz;  // d/dt
  R exx, exy, exz, bxy, bxz;  // d/dx
};

template <typename R>
struct MomentumOut {
  R Lx, Ly, Lz;     // u_L^{n+1/2}, after the Boris step
  R nx, ny, nz;     // u^{n+1/2} as stored
  R ddx, ddy, ddz;  // the RR increment added (with the carried residual under COMP)
  R gL;             // gamma of u_L (RR only)
};

// One momentum step of the paper's scheme (Section 3): Boris for the Lorentz
// force (Eq. (part1)), then the RR increment dt f_R of Eq. (f_r) at the
// mid-step estimate p^(n) = (u_L + u^{n-1/2}) / 2 of Eqs. (estim1) and
// (estimgamma), added as in Eq. (pertfull).  qh = q dt / (2 m), k = eps dt.
// COMP adds the increment by TwoSum and carries the FP32 rounding residual
// in (rx, ry, rz).  DERIV adds the derivative term of Eq. (3dLL) at the same
// p^(n) (the complete LL force, for tracking in given fields).  BX takes a
// non-zero B_x (multi-dimensional grids); without it B_x = 0, as in 1D, and
// none of its terms is evaluated.
template <typename R, bool RR, bool COMP, bool DERIV, bool BX = false>
__device__ __forceinline__ void momentum_step(R ux, R uy, R uz, R ex, R ey, R ez, R by, R bz, R qh,
                                              R k, const FieldRates<R>& fr, float& rx, float& ry,
                                              float& rz, float& stiff, MomentumOut<R>& o,
                                              R bx = R(0)) {
  // Boris
  const R hx = qh * ex, hy = qh * ey, hz = qh * ez;
  const R mx = ux + hx, my = uy + hy, mz = uz + hz;
  const R igm = rsq(R(1) + mx * mx + my * my + mz * mz);
  const R ty = qh * by * igm, tz = qh * bz * igm;
  R tx = R(0), den;
  if constexpr (BX) {
    tx = qh * bx * igm;
    den = R(1) + tx * tx + ty * ty + tz * tz;
  } else {
    den = R(1) + ty * ty + tz * tz;
  }
  const R sf = R(2) * rcp(den);
  R px = mx + (my * tz - mz * ty);
  R py = my - mx * tz;
  R pz = mz + mx * ty;
  if constexpr (BX) {
    py += mz * tx;
    pz -= my * tx;
  }
  const R sy = sf * ty, sz = sf * tz;
  R Lx = mx + (py * sz - pz * sy) + hx;
  R Ly = my - px * sz + hy;
  R Lz = mz + px * sy + hz;
  if constexpr (BX) {
    const R sx = sf * tx;
    Ly += pz * sx;
    Lz -= py * sx;
  }

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
    R Fy = ey - vx * bz;
    R Fz = ez + vx * by;
    if constexpr (BX) {
      Fy += vz * bx;
      Fz -= vy * bx;
    }
    const R vE = vx * ex + vy * ey + vz * ez;
    R br = Fx * Fx + Fy * Fy + Fz * Fz - vE * vE;
    br = br > R(0) ? br : R(0);
    const R g2b = g2 * br;
    // dt f_R = dt eps [F x B + (v.E) E - gamma^2 (F^2 - (v.E)^2) v]
    if constexpr (BX) {
      ddx = k * ((Fy * bz - Fz * by) + vE * ex - g2b * vx);
      ddy = k * ((Fz * bx - Fx * bz) + vE * ey - g2b * vy);
      ddz = k * ((Fx * by - Fy * bx) + vE * ez - g2b * vz);
    } else {
      ddx = k * ((Fy * bz - Fz * by) + vE * ex - g2b * vx);
      ddy = k * (vE * ey - Fx * bz - g2b * vy);
      ddz = k * (Fx * by + vE * ez - g2b * vz);
    }
    if (DERIV) {
      // derivative term of Eq. (3dLL): -eps gamma [D E + v x D B], D = d/dt + v_x d/dx
      const R g = g2 * ig;
      const R DEx = fr.etx + vx * fr.exx, DEy = fr.ety + vx * fr.exy, DEz = fr.etz + vx * fr.exz;
      const R DBy = fr.bty + vx * fr.bxy, DBz = fr.btz + vx * fr.bxz;
      ddx -= k * g * (DEx + (vy * DBz - vz * DBy));
      ddy -= k * g * (DEy - vx * DBz);
      ddz -= k * g * (DEz + vx * DBy);
    }
    if (ddx * ddx + ddy * ddy + ddz * ddz > R(0.01) * (Lx * Lx + Ly * Ly + Lz * Lz)) stiff += 1.f;
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
    gL = fsqrt(R(1) + Lx * Lx + Ly * Ly + Lz * Lz);
  }

  o.Lx = Lx;
  o.Ly = Ly;
  o.Lz = Lz;
  o.nx = nx;
  o.ny = ny;
  o.nz = nz;
  o.ddx = ddx;
  o.ddy = ddy;
  o.ddz = ddz;
  o.gL = gL;
}

// All loads of one particle are independent of each other, so a thread keeps
// several particles' loads in flight while it computes an earlier one.
// Past the end of the species (i >= n, last tile only) the loads read
// particle n - 1 instead, so that they need no branch, and the particle is
// marked removed.  n >= 1.
template <typename R, bool COMP>
__device__ __forceinline__ PData<R> load_particle(const SpeciesDev<R>& sp, int i, int n) {
  PData<R> d;
  const bool in = i < n;
  const unsigned ui = (unsigned)(in ? i : n - 1);
  d.c = ld(sp.cell, ui);
  if (!in) d.c = kDead;
  d.o = ld(sp.off, ui);
  d.ux = ld(sp.ux, ui);
  d.uy = ld(sp.uy, ui);
  d.uz = ld(sp.uz, ui);
  d.w = ld(sp.w, ui);
  if (COMP) {
    d.rx = ld(sp.rx, ui);
    d.ry = ld(sp.ry, ui);
    d.rz = ld(sp.rz, ui);
  } else {
    d.rx = d.ry = d.rz = 0.f;
  }
  return d;
}

// The four field loads of one particle's gather: (E_y, E_z) at the nodes
// either side and (E_x, B_y, B_z) at the half-nodes either side.  They are
// issued from the particle's ring entry one particle ahead of its push, so
// that their latency overlaps the push of the particle before it.
template <typename R>
struct Gath {
  NodeF<R> n0, n1;
  HalfF<R> h0, h1;
};

template <typename R>
__device__ __forceinline__ Gath<R> gather_issue(const FieldsDev<R>& f, const PData<R>& pd) {
  const unsigned uc = pd.c == kDead ? 0u : (unsigned)pd.c;  // removed: any valid address
  const unsigned h = uc + (pd.o + R(0.5) >= R(1));
  Gath<R> g;
  g.n0 = ld(f.N, uc);
  g.n1 = ld(f.N, uc + 1);
  g.h0 = ld(f.H, h);
  g.h1 = ld(f.H, h + 1);
  return g;
}

// One particle: gather (from its field loads issued ahead), Boris, RR, move,
// deposit, store.
template <typename R, bool RR, bool COMP>
__device__ __forceinline__ void push_particle(const PushArgs<R>& a, const SpeciesDev<R>& sp,
                                              int s, int i, const PData<R>& pd, const Gath<R>& gf,
                                              DepositCtx& dc, PushAcc& acc) {
  const int c = pd.c;
  if (c == kDead) return;
  const unsigned ui = (unsigned)i;
  const R o = pd.o, ux = pd.ux, uy = pd.uy, uz = pd.uz, w = pd.w;
  float rx = pd.rx, ry = pd.ry, rz = pd.rz;

  // ---- gather E^n, B^n (linear weights; E_y,E_z on nodes, the rest on half-nodes).
  // The fused multiply-adds are written out: left to contraction, the two
  // unrolled ring slots were compiled with different roundings, and a
  // particle's result then depended on its slot, which the sort's order
  // within a cell leaves open.
  const R on = R(1) - o;
  const NodeF<R> n0 = gf.n0, n1 = gf.n1;
  const R ey = fma(o, n1.ey, on * n0.ey);
  const R ez = fma(o, n1.ez, on * n0.ez);
  const R sx = o + R(0.5);
  const unsigned hb = sx >= R(1);
  const R fh = hb ? sx - R(1) : sx;
  const R fn = R(1) - fh;
  const HalfF<R> h0 = gf.h0, h1 = gf.h1;
  const R ex = fma(fh, h1.ex, fn * h0.ex);
  const R by = fma(fh, h1.by, fn * h0.by);
  const R bz = fma(fh, h1.bz, fn * h0.bz);

  MomentumOut<R> mo;
  momentum_step<R, RR, COMP, false>(ux, uy, uz, ex, ey, ez, by, bz, a.qh[s], a.eps * a.dt,
                                    FieldRates<R>{}, rx, ry, rz, acc.stiff, mo);
  const R Lx = mo.Lx, Ly = mo.Ly, Lz = mo.Lz;
  const R nx = mo.nx, ny = mo.ny, nz = mo.nz;
  const R ddx = mo.ddx, ddy = mo.ddy, ddz = mo.ddz, gL = mo.gL;

  // ---- move (contract arithmetic)
  R g, vy, vz, o1, shift;
  contract_move<R>(nx, ny, nz, o, a.cfl, g, vy, vz, o1, shift);
  if (!(fabs(shift) < R(4)) || !(g < R(1e30))) {  // NaN/Inf momentum: drop it, raise the flag
    st(sp.cell, ui, kDead);
    atomicOr(a.flags, 1);
    return;
  }
  const int c1 = c + (int)shift;
  const int qw = a.Z[s] * (int)rint(w * a.sw);
  deposit<R>(dc, c, o, c1, o1, vy, vz, qw);

  if (RR) {
    // gamma_L - gamma_new = -(d . (2 u_L + d)) / (gamma_L + gamma_new)
    const R num = ddx * (R(2) * Lx + ddx) + ddy * (R(2) * Ly + ddy) + ddz * (R(2) * Lz + ddz);
    acc.rad -= (float)(w * num * rcp(gL + g));
  }
  if (c1 < 0 || c1 >= a.nx) {
    st(sp.cell, ui, kDead);
    acc.esc += (float)(w * (R)a.mass[s] * (g - R(1)));
  } else {
    st(sp.cell, ui, c1);
    st(sp.off, ui, o1);
    acc.cmin1 = min(acc.cmin1, c1);
    acc.cmax1 = max(acc.cmax1, c1);
  }
  st(sp.ux, ui, nx);
  st(sp.uy, ui, ny);
  st(sp.uz, ui, nz);
  if (COMP) {
    st(sp.rx, ui, rx);
    st(sp.ry, ui, ry);
    st(sp.rz, ui, rz);
  }
}

// PPT particles per thread, D of them with loads in flight (D = PPT: the
// whole tile is loaded up front)
template <typename R, bool RR, bool COMP, int PPT, int D>
__device__ __forceinline__ void push_tile(const PushArgs<R>& a, int s, int tile, int n, int base,
                                          unsigned long long* lds) {
  static_assert(PPT % D == 0, "the load ring must divide the tile");
  // the next particle's field loads are issued from its ring entry, which
  // must be a different entry from the current particle's
  static_assert(D >= 2 || PPT == 1, "a ring of one entry holds one particle per thread only");
  __shared__ int s_mn[kThreads / kLanes], s_mx[kThreads / kLanes];
  __shared__ double s_red[3][kThreads / kLanes];
  const SpeciesDev<R> sp = a.sp[s];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

  // the first particles' loads overlap the window set-up below
  PData<R> ring[D];
#pragma unroll
  for (int k = 0; k < D; ++k) ring[k] = load_particle<R, COMP>(sp, base + k * kThreads + tid, n);

  // the tile's cell range: as the previous push left it, when that is
  // known, else from a pass over the cells (from the ring when it holds the
  // whole tile)
  int cmin = INT_MAX, cmax = INT_MIN;
  if (__builtin_amdgcn_readfirstlane(*a.pred_in)) {
    cmin = __builtin_amdgcn_readfirstlane(a.rng_in[2 * tile]);
    cmax = __builtin_amdgcn_readfirstlane(a.rng_in[2 * tile + 1]);
  } else {
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      int c;
      if constexpr (PPT == D) {
        c = ring[k].c;
      } else {
        const int i = base + k * kThreads + tid;
        c = i < n ? ld(sp.cell, (unsigned)i) : kDead;
      }
      if (c != kDead) {
        cmin = min(cmin, c);
        cmax = max(cmax, c);
      }
    }
    cmin = wave_min_dpp(cmin);
    cmax = wave_max_dpp(cmax);
    if (lane == 0) {
      s_mn[wid] = cmin;
      s_mx[wid] = cmax;
    }
    __syncthreads();
    cmin = min(min(s_mn[0], s_mn[1]), min(s_mn[2], s_mn[3]));
    cmax = max(max(s_mx[0], s_mx[1]), max(s_mx[2], s_mx[3]));
  }
  if (cmin > cmax) {  // every particle of the tile was removed
    if (tid == 0) {
      a.rng_out[2 * tile] = INT_MAX;
      a.rng_out[2 * tile + 1] = INT_MIN;
      *a.pred_out = 1;
    }
    return;
  }

  // window: storage indices cmin .. cmax + 3 (nodes cmin - 1 .. cmax + 2),
  // with as many private copies per slot (up to 64) as the LDS holds
  DepositCtx dc;
  dc.lds = lds;
  dc.J[0] = a.J[0];
  dc.J[1] = a.J[1];
  dc.J[2] = a.J[2];
  dc.wlo = cmin;
  dc.W = cmax - cmin + 4;
  dc.qw_ref = a.qw_ref[s];
  int sh = 6;
  while (sh > 0 && 3 * dc.W * ((1 << sh) + 1) > kLdsSlots) --sh;
  dc.P = sh ? (1 << sh) + 1 : 1;
  dc.copy = lane & ((1 << sh) - 1);
  const int E = 3 * dc.W * dc.P;
  dc.use_lds = E <= kLdsSlots;
  if (dc.use_lds)
    for (int e = tid; e < E; e += kThreads) lds[e] = 0ull;
  __syncthreads();

  PushAcc acc{0.f, 0.f, 0.f, INT_MAX, INT_MIN};
  // ring slot j holds particle k0 + j; its successor D ahead is loaded
  // before particle k0 + j is computed, and the field loads of particle
  // k0 + j + 1 (whose ring entry has arrived) before those of k0 + j + D
  Gath<R> gnext = gather_issue<R>(a.f, ring[0]);
#pragma unroll kRingUnroll
  for (int k0 = 0; k0 < PPT; k0 += D) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int i = base + (k0 + j) * kThreads + tid;
      const PData<R> cur = ring[j];
      const Gath<R> gcur = gnext;
      if (k0 + j + 1 < PPT) gnext = gather_issue<R>(a.f, ring[(j + 1) % D]);
      if (k0 + j + D < PPT) ring[j] = load_particle<R, COMP>(sp, i + D * kThreads, n);
      push_particle<R, RR, COMP>(a, sp, s, i, cur, gcur, dc, acc);
    }
  }

  const double r0 = wave_sum_dpp((double)acc.rad), r1 = wave_sum_dpp((double)acc.esc),
               r2 = wave_sum_dpp((double)acc.stiff);
  const int n0 = wave_min_dpp(acc.cmin1), n1 = wave_max_dpp(acc.cmax1);
  if (lane == 0) {
    s_red[0][wid] = r0;
    s_red[1][wid] = r1;
    s_red[2][wid] = r2;
    s_mn[wid] = n0;
    s_mx[wid] = n1;
  }
  __syncthreads();

  // flush: g lanes per slot each sum R / g copies, DPP adds the g partial
  // sums, and the group's last lane issues one global atomic
  if (dc.use_lds) {
    const int nc = 1 << sh;  // copies per slot
    const int gsh = sh < 4 ? sh : 4, g = 1 << gsh;
    const int S = 3 * dc.W, gi = tid >> gsh, t = tid & (g - 1);
    for (int s0 = 0; s0 < S; s0 += kThreads >> gsh) {
      const int sl = s0 + gi;
      long long v = 0;
      if (sl < S) {
        const unsigned long long* q = lds + sl * dc.P + t;
        for (int k = 0; k < nc; k += g) v += (long long)q[k];
      }
      v = group_sum(v, g);
      if (t == g - 1 && sl < S && v != 0) {
        const int comp = sl / dc.W, j = sl - comp * dc.W;
        atomicAdd(a.J[comp] + dc.wlo + j, (unsigned long long)(v * (long long)dc.qw_ref));
      }
    }
  }
  if (tid == 0) {
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int w = 0; w < kThreads / kLanes; ++w) {
      t0 += s_red[0][w];
      t1 += s_red[1][w];
      t2 += s_red[2][w];
    }
    // the tile's cells for the next push
    a.rng_out[2 * tile] = min(min(s_mn[0], s_mn[1]), min(s_mn[2], s_mn[3]));
    a.rng_out[2 * tile + 1] = max(max(s_mx[0], s_mx[1]), max(s_mx[2], s_mx[3]));
    *a.pred_out = 1;
    // one add per slot and launch, in launch order: deterministic; the
    // atomic form needs no load, so the work-group retires without waiting
    double* A = a.acc + 4 * (size_t)tile;
    unsafeAtomicAdd(A + 0, t0);
    unsafeAtomicAdd(A + 1 + s, t1);
    unsafeAtomicAdd(A + 3, t2);
  }
}

template <typename R, int PPT, int D>
__device__ __forceinline__ void push_one_tile(const PushArgs<R>& a, int tile,
                                              unsigned long long* lds) {
  const int s = tile < a.tiles0 ? 0 : 1;
  const int tl = s ? tile - a.tiles0 : tile;
  const int n = (int)a.count[s];
  const int base = tl * (kThreads * PPT);
  if (base >= n) return;
  if (s == 0 && a.rr0) {
    if (a.comp)
      push_tile<R, true, true, PPT, D>(a, s, tile, n, base, lds);
    else
      push_tile<R, true, false, PPT, D>(a, s, tile, n, base, lds);
  } else {
    push_tile<R, false, false, PPT, D>(a, s, tile, n, base, lds);
  }
}

#if PIC_PUSH_MIN_WAVES > 0
#define PIC_PUSH_BOUNDS __launch_bounds__(kThreads, PIC_PUSH_MIN_WAVES)
#else
#define PIC_PUSH_BOUNDS __launch_bounds__(kThreads)
#endif

// one work-group per tile
template <typename R>
__global__ PIC_PUSH_BOUNDS void k_push(PushArgs<R> a) {
  __shared__ unsigned long long lds[kLdsSlots];
  push_one_tile<R, kPPT, kDepth>(a, a.tile0 + (int)blockIdx.x, lds);
}

// the same push in tiles of kBatchTile (two particles' loads in flight, as
// in the batched push), for runs too small to fill the device with kTile tiles
template <typename R>
__global__ PIC_PUSH_BOUNDS void k_push_small(PushArgs<R> a) {
  __shared__ unsigned long long lds[kLdsSlots];
  push_one_tile<R, kBatchPPT, kBatchDepth>(a, a.tile0 + (int)blockIdx.x, lds);
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
  int tick;                       // 1: work-group 0 advances *step after the update
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

// LDS elements of a field chunk of CH nodes
template <int CH>
constexpr int field_lds_elems() { return 8 * CH + 14; }

// One chunk of CH nodes (the work-group has CH threads).  `ahead` is the
// number of steps the run is past its device step counter (a launch that
// advances several steps before the counter moves); `sm` holds
// field_lds_elems<CH>() elements of LDS.
template <typename R, int CH>
__device__ __forceinline__ void field_chunk(const FieldArgs<R>& p, int chunk, int ahead, R* sm) {
  R* sEy = sm;                    // E^n, nodes i0-2 .. i0+CH
  R* sEz = sEy + (CH + 3);
  R* sBy = sEz + (CH + 3);        // B, half-nodes i0-1 .. i0+CH
  R* sBz = sBy + (CH + 2);
  R* sJy = sBz + (CH + 2);        // J, nodes i0-1 .. i0+CH-1
  R* sJz = sJy + (CH + 1);
  R* nEy = sJz + (CH + 1);        // E^{n+1}, nodes i0-1 .. i0+CH-1
  R* nEz = nEy + (CH + 1);
  const int t = threadIdx.x;
  const int i0 = chunk * CH;
  const int n = p.nx;
  const R a = p.a, ha = R(0.5) * p.a, dt = p.dt;

  // loads needed only at the end are issued first, so that their latency
  // overlaps the staged update below
  const int h = i0 + t;  // this thread's half-node (and node) output
  long long ex_old = 0, jx = 0;
  if (h <= n + 1) {
    ex_old = p.Ex_int[h];
    jx = p.J[0][h];
  }
  // incident wave at t_{n+1/2} (work-group 0 only)
  double ey_in = 0.0, ez_in = 0.0;
  if (t == 0 && i0 == 0) {
    const double th = ((double)(*p.step + ahead) + 0.5) * p.dtd;
    const double f = envelope(th, p.tr, p.tf, p.tl);
    ey_in = p.ay * f * sin(th);
    ez_in = p.az * f * cos(th);
  }

  for (int k = t; k < CH + 3; k += CH) {
    const int i = i0 - 2 + k;
    const bool ok = i >= 0 && i <= n;
    const NodeF<R> v = ok ? p.in.N[i] : NodeF<R>{R(0), R(0)};
    sEy[k] = v.ey;
    sEz[k] = v.ez;
  }
  for (int k = t; k < CH + 2; k += CH) {
    const int h = i0 - 1 + k;
    const bool ok = h >= 0 && h <= n + 1;
    const HalfF<R> v = ok ? p.in.H[h] : HalfF<R>{R(0), R(0), R(0), R(0)};
    sBy[k] = v.by;
    sBz[k] = v.bz;
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
  if (t == 0 && i0 == 0) {
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
    if (p.tick) *p.step += 1;
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
    p.out.N[i] = NodeF<R>{nEy[t + 1], nEz[t + 1]};
  }
  if (h <= n + 1) {
    R bz, byv;
    if (h >= 1 && h <= n) {  // B^{n+1/2} -> B^{n+1}
      bz = sBz[t + 1] - ha * (nEy[t + 1] - nEy[t]);
      byv = sBy[t + 1] + ha * (nEz[t + 1] - nEz[t]);
    } else {                 // guards keep their t_{n+1/2} value
      bz = sBz[t + 1];
      byv = sBy[t + 1];
    }
    const long long ex = ex_old - jx;
    p.Ex_int[h] = ex;
    p.out.H[h] = HalfF<R>{(R)((double)ex * p.sEx), byv, bz, R(0)};
    p.Jnext[0][h] = 0ull;
  }
  if (i0 + t <= n + 2) {
    p.Jnext[1][i0 + t] = 0ull;
    p.Jnext[2][i0 + t] = 0ull;
  }
}

template <typename R>
__global__ __launch_bounds__(kFieldChunk) void k_field(FieldArgs<R> p) {
  __shared__ R sm[field_lds_elems<kFieldChunk>()];
  field_chunk<R, kFieldChunk>(p, (int)blockIdx.x, 0, sm);
}

// ---------------------------------------------------------------- sort
template <typename R>
struct SortArgs {
  SpeciesDev<R> src[2], dst[2];
  const long long* count;  // [2] particles in the source arrays
  int* cnt[2];          // [n] per-cell counts (zero on entry to k_sort_hist)
  int* cursor[2];       // [n] scatter cursors
  int blocks0;          // blocks of species 0 in hist / scatter grids
  int blk0;             // first block of this launch (a pass may be split over launches)
  int nx;
  int comp;             // carry residuals of species 0
  int* pred;            // [2] the push's range-prediction flags, cleared: the order changes
  int ysh, bxs, bys;    // 2D grids: cell = ix << ysh | iy, sorted by blocks of 2^bxs x 2^bys cells
};

// Sort key of a 2D cell: blocks of 2^bxs x 2^bys cells column by column,
// and the cells of a block column by column, so that the particles of a
// sort tile (and of a push tile) lie in a compact patch of the grid rather
// than along one column.  A bijection of [0, roundup(nx, 2^bxs) << ysh);
// with bxs = bys = 0 the key is the cell index itself.
__device__ __forceinline__ int sort_key2(int c, int ysh, int bxs, int bys) {
  if (c == kDead) return kDead;
  const int ix = c >> ysh, iy = c & ((1 << ysh) - 1);
  return ((ix >> bxs) << (ysh + bxs)) | ((iy >> bys) << (bxs + bys)) |
         ((ix & ((1 << bxs) - 1)) << bys) | (iy & ((1 << bys) - 1));
}

constexpr int kSortThreads = 256;
constexpr int kSortPPT = 8;                        // particles per thread per sort tile
constexpr int kSortTile = kSortThreads * kSortPPT;
constexpr int kSortWin = 4096;                     // LDS cell window of a sort tile

// wave-aggregated atomicAdd(ptr[key], 1) returning each lane's slot: one
// atomic per distinct key in the wave (ptr may point to LDS or HBM)
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

// Cell range of a sort tile (block-uniform result).
__device__ __forceinline__ void tile_range(const int* cl, int& lo, int& hi, int* sm) {
  int a = INT_MAX, b = INT_MIN;
#pragma unroll
  for (int k = 0; k < kSortPPT; ++k)
    if (cl[k] != kDead) {
      a = min(a, cl[k]);
      b = max(b, cl[k]);
    }
  a = wave_min_dpp(a);
  b = wave_max_dpp(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();  // earlier readers of sm (previous tile) are done
  if (lane == 0) {
    sm[wid] = a;
    sm[4 + wid] = b;
  }
  __syncthreads();
  lo = min(min(sm[0], sm[1]), min(sm[2], sm[3]));
  hi = max(max(sm[4], sm[5]), max(sm[6], sm[7]));
}

// per-cell particle counts: LDS histogram over the tile's cell window,
// then one global atomic per occupied cell and tile
template <typename R, bool KEY2 = false>
__device__ __forceinline__ void sort_hist_block(const SortArgs<R>& p, int blk) {
  __shared__ int cnt[kSortWin];
  __shared__ int sm[8];
  const int s = blk < p.blocks0 ? 0 : 1;
  const int b = s ? blk - p.blocks0 : blk;
  const long long n = p.count[s];
  const long long base = (long long)b * kSortTile;
  if (base >= n) return;
  int cl[kSortPPT];
#pragma unroll
  for (int k = 0; k < kSortPPT; ++k) {
    const long long i = base + k * kSortThreads + threadIdx.x;
    cl[k] = i < n ? p.src[s].cell[i] : kDead;
    if constexpr (KEY2) cl[k] = sort_key2(cl[k], p.ysh, p.bxs, p.bys);
  }
  int lo, hi;
  tile_range(cl, lo, hi, sm);
  if (lo > hi) return;
  const int W = hi - lo + 1;
  if (W <= kSortWin) {
    for (int e = threadIdx.x; e < W; e += kSortThreads) cnt[e] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortPPT; ++k) wave_claim(cnt, cl[k] - lo, cl[k] != kDead);
    __syncthreads();
    for (int e = threadIdx.x; e < W; e += kSortThreads)
      if (cnt[e]) atomicAdd(p.cnt[s] + lo + e, cnt[e]);
  } else {
#pragma unroll
    for (int k = 0; k < kSortPPT; ++k) wave_claim(p.cnt[s], cl[k], cl[k] != kDead);
  }
}

template <typename R>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(SortArgs<R> p) {
  sort_hist_block<R>(p, p.blk0 + (int)blockIdx.x);
}

// inclusive prefix sum over the 64 lanes of a wave (all lanes active)
__device__ __forceinline__ int wave_incl_scan(int v) {
  v += row_shr<1>(0, v);
  v += row_shr<2>(0, v);
  v += row_shr<4>(0, v);
  v += row_shr<8>(0, v);
  const int r0 = __builtin_amdgcn_readlane(v, 15), r1 = __builtin_amdgcn_readlane(v, 31),
            r2 = __builtin_amdgcn_readlane(v, 47);
  const int row = (threadIdx.x & 63) >> 4;
  return v + (row >= 1 ? r0 : 0) + (row >= 2 ? r1 : 0) + (row >= 3 ? r2 : 0);
}

// Exclusive scan of one chunk of kScanChunk per-cell counts (one work-group
// of 1024 threads), starting from `carry`: the chunk passes through LDS so
// that every global access is coalesced; within it thread t scans cells
// 8t .. 8t + 7.  Writes the cursors, clears the counts for the next
// histogram and returns the chunk's total.
constexpr int kScanThreads = 1024, kScanPer = 8, kScanChunk = kScanThreads * kScanPer;
__device__ __forceinline__ int scan_chunk(int* cnt, int* cur, int c0, int nx, long long carry,
                                          int* stage, int* wsum) {
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int j = c0 + k * kScanThreads + t;
    stage[k * kScanThreads + t] = j < nx ? cnt[j] : 0;
  }
  __syncthreads();
  int v[kScanPer], sum = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = stage[t * kScanPer + k];
    sum += v[k];
  }
  const int incl = wave_incl_scan(sum);
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int before = 0, total = 0;
  for (int w = 0; w < kScanThreads / kLanes; ++w) {
    before += w < wid ? wsum[w] : 0;
    total += wsum[w];
  }
  int run = (int)carry + before + incl - sum;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    stage[t * kScanPer + k] = run;
    run += v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int j = c0 + k * kScanThreads + t;
    if (j < nx) {
      cur[j] = stage[k * kScanThreads + t];
      cnt[j] = 0;
    }
  }
  __syncthreads();  // stage and wsum are reused by the next chunk
  return total;
}

// exclusive scan of the per-cell counts of one species in one work-group,
// chunk after chunk; the alive count goes to *new_count (the count slot of
// the destination arrays)
__device__ __forceinline__ void sort_scan_species(int* cnt, int* cur, long long* new_count, int nx) {
  __shared__ int stage[kScanChunk];
  __shared__ int wsum[kScanThreads / kLanes];
  long long carry = 0;
  for (int c0 = 0; c0 < nx; c0 += kScanChunk) carry += scan_chunk(cnt, cur, c0, nx, carry, stage, wsum);
  if (threadIdx.x == 0) *new_count = carry;
}

__global__ __launch_bounds__(1024) void k_sort_scan(int* cnt0, int* cnt1, int* cur0, int* cur1,
                                                    long long* new_count, int nx) {
  if (blockIdx.x == 0)
    sort_scan_species(cnt0, cur0, new_count, nx);
  else
    sort_scan_species(cnt1, cur1, new_count + 1, nx);
}

// scatter to the destination arrays: each tile claims, per occupied cell,
// one contiguous range of the cell's bucket with a single global atomic and
// hands out positions inside it through an LDS counter (OY: particles of a
// 2D grid also carry a y offset)
template <typename R, bool OY = false>
__device__ __forceinline__ void sort_scatter_block(const SortArgs<R>& p, int blk) {
  __shared__ int cnt[kSortWin];
  __shared__ int sm[8];
  const int s = blk < p.blocks0 ? 0 : 1;
  const int b = s ? blk - p.blocks0 : blk;
  const long long n = p.count[s];
  const long long base = (long long)b * kSortTile;
  if (blk == 0 && threadIdx.x == 0) p.pred[0] = p.pred[1] = 0;
  if (base >= n) return;
  const SpeciesDev<R> src = p.src[s], dst = p.dst[s];
  const bool comp = s == 0 && p.comp;
  int cl[kSortPPT], pos[kSortPPT];
  // the particles' data is loaded with their cells, so that its latency
  // overlaps the position claims below
  R off[kSortPPT], ux[kSortPPT], uy[kSortPPT], uz[kSortPPT], w[kSortPPT], oy[kSortPPT];
  float rx[kSortPPT], ry[kSortPPT], rz[kSortPPT];
#pragma unroll
  for (int k = 0; k < kSortPPT; ++k) {
    const long long i = base + k * kSortThreads + threadIdx.x;
    cl[k] = kDead;
    if (i < n) {
      const unsigned ui = (unsigned)i;
      cl[k] = ld(src.cell, ui);
      off[k] = ld(src.off, ui);
      ux[k] = ld(src.ux, ui);
      uy[k] = ld(src.uy, ui);
      uz[k] = ld(src.uz, ui);
      w[k] = ld(src.w, ui);
      if constexpr (OY) oy[k] = ld(src.oy, ui);
      if (comp) {
        rx[k] = ld(src.rx, ui);
        ry[k] = ld(src.ry, ui);
        rz[k] = ld(src.rz, ui);
      }
    }
  }
  // bucket keys: the cell itself, or its 2D block key (OY)
  int ky[kSortPPT];
#pragma unroll
  for (int k = 0; k < kSortPPT; ++k) {
    if constexpr (OY) ky[k] = sort_key2(cl[k], p.ysh, p.bxs, p.bys);
    else ky[k] = cl[k];
  }
  int lo, hi;
  tile_range(ky, lo, hi, sm);
  if (lo > hi) return;
  const int W = hi - lo + 1;
  if (W <= kSortWin) {
    for (int e = threadIdx.x; e < W; e += kSortThreads) cnt[e] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortPPT; ++k) pos[k] = wave_claim(cnt, ky[k] - lo, ky[k] != kDead);
    __syncthreads();
    for (int e = threadIdx.x; e < W; e += kSortThreads)
      cnt[e] = cnt[e] ? atomicAdd(p.cursor[s] + lo + e, cnt[e]) : 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortPPT; ++k)
      if (ky[k] != kDead) pos[k] += cnt[ky[k] - lo];
  } else {
#pragma unroll
    for (int k = 0; k < kSortPPT; ++k) pos[k] = wave_claim(p.cursor[s], ky[k], ky[k] != kDead);
  }
#pragma unroll
  for (int k = 0; k < kSortPPT; ++k) {
    if (cl[k] == kDead) continue;
    const unsigned j = (unsigned)pos[k];
    st(dst.cell, j, cl[k]);
    st(dst.off, j, off[k]);
    st(dst.ux, j, ux[k]);
    st(dst.uy, j, uy[k]);
    st(dst.uz, j, uz[k]);
    st(dst.w, j, w[k]);
    if constexpr (OY) st(dst.oy, j, oy[k]);
    if (comp) {
      st(dst.rx, j, rx[k]);
      st(dst.ry, j, ry[k]);
      st(dst.rz, j, rz[k]);
    }
  }
}

template <typename R>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(SortArgs<R> p) {
  sort_scatter_block<R>(p, p.blk0 + (int)blockIdx.x);
}

// ---------------------------------------------------------------- test electrons
// Independent electrons in a given monochromatic plane wave travelling along
// +x (the single-particle tests of Section 3): A_y = a_y sin(phi + psi),
// A_z = a_z cos(phi + psi), phi = t - x, E_perp = -dA/dphi, B = (0, -E_z, E_y).
struct TrackArgs {
  double ay, az, psi;
  double dt, t0;
  double eps;
  long long steps, n;
  double* x;
  double* ux;
  double* uy;
  double* uz;
};

// Fields (and, for the complete force, their partial derivatives) at (x, t)
template <typename R>
__device__ __forceinline__ void wave_at(const TrackArgs& a, double x, double t, R& ey, R& ez,
                                        FieldRates<R>& fr) {
  double sn, cs;
  sincos(t - x + a.psi, &sn, &cs);
  ey = (R)(-a.ay * cs);
  ez = (R)(a.az * sn);
  // dE_perp/dphi = (a_y sin, a_z cos); d/dt = d/dphi, d/dx = -d/dphi
  const R dy = (R)(a.ay * sn), dz = (R)(a.az * cs);
  fr.etx = R(0);
  fr.ety = dy;
  fr.etz = dz;
  fr.bty = -dz;
  fr.btz = dy;
  fr.exx = R(0);
  fr.exy = -dy;
  fr.exz = -dz;
  fr.bxy = dz;
  fr.bxz = -dy;
}

// The paper's leapfrog scheme: x^n and u^{n-1/2} in, x^{n+steps} and
// u^{n+steps-1/2} out; the position advances in FP64 by dt u_x / gamma.
// MODE: 0 Lorentz only, 1 with f_R of Eq. (f_r), 2 with the complete force.
template <typename R, int MODE>
__global__ void k_track_leapfrog(TrackArgs a) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  constexpr bool COMP = sizeof(R) == 4 && MODE > 0;
  double x = a.x[i];
  R ux = (R)a.ux[i], uy = (R)a.uy[i], uz = (R)a.uz[i];
  float rx = 0.f, ry = 0.f, rz = 0.f, stiff = 0.f;
  const R qh = (R)(-0.5 * a.dt), k = (R)(a.eps * a.dt);
  for (long long s = 0; s < a.steps; ++s) {
    R ey, ez;
    FieldRates<R> fr;
    wave_at<R>(a, x, a.t0 + (double)s * a.dt, ey, ez, fr);
    MomentumOut<R> o;
    momentum_step<R, (MODE > 0), COMP, (MODE == 2)>(ux, uy, uz, R(0), ey, ez, -ez, ey, qh, k, fr, rx,
                                                    ry, rz, stiff, o);
    ux = o.nx;
    uy = o.ny;
    uz = o.nz;
    const double gx = (double)ux + rx, gy = (double)uy + ry, gz = (double)uz + rz;
    x += a.dt * gx / sqrt(1.0 + gx * gx + gy * gy + gz * gz);
  }
  a.x[i] = x;
  a.ux[i] = (double)ux + rx;
  a.uy[i] = (double)uy + ry;
  a.uz[i] = (double)uz + rz;
}

// Right-hand side of Eq. (3dLL) for an electron (MODE 0: Lorentz only; 1:
// plus the non-derivative RR terms; 2: plus the derivative term).
template <typename R, int MODE>
__device__ __forceinline__ void ll_rhs(R ux, R uy, R uz, R ey, R ez, const FieldRates<R>& fr, R eps,
                                       R& fx, R& fy, R& fz) {
  const R by = -ez, bz = ey;
  const R g2 = R(1) + ux * ux + uy * uy + uz * uz;
  const R ig = R(1) / sqrt(g2);
  const R vx = ux * ig, vy = uy * ig, vz = uz * ig;
  const R Fx = vy * bz - vz * by, Fy = ey - vx * bz, Fz = ez + vx * by;  // E + v x B (E_x = 0)
  fx = -Fx;
  fy = -Fy;
  fz = -Fz;
  if (MODE > 0) {
    const R vE = vy * ey + vz * ez;
    const R br = g2 * (Fx * Fx + Fy * Fy + Fz * Fz - vE * vE);
    fx += eps * ((Fy * bz - Fz * by) - br * vx);
    fy += eps * (vE * ey - Fx * bz - br * vy);
    fz += eps * (Fx * by + vE * ez - br * vz);
  }
  if (MODE == 2) {
    const R g = g2 * ig;
    const R DEy = fr.ety + vx * fr.exy, DEz = fr.etz + vx * fr.exz;
    const R DBy = fr.bty + vx * fr.bxy, DBz = fr.btz + vx * fr.bxz;
    fx -= eps * g * (vy * DBz - vz * DBy);
    fy -= eps * g * (DEy - vx * DBz);
    fz -= eps * g * (DEz + vx * DBy);
  }
}

// Classical RK4 of (x, u) at the same time, the comparator of Section 3.
template <typename R, int MODE>
__global__ void k_track_rk4(TrackArgs a) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  double x = a.x[i];
  R ux = (R)a.ux[i], uy = (R)a.uy[i], uz = (R)a.uz[i];
  const R h = (R)a.dt, eps = (R)a.eps;
  auto stage = [&](double xs, double ts, R sx, R sy, R sz, double& dx, R& fx, R& fy, R& fz) {
    R ey, ez;
    FieldRates<R> fr;
    wave_at<R>(a, xs, ts, ey, ez, fr);
    ll_rhs<R, MODE>(sx, sy, sz, ey, ez, fr, eps, fx, fy, fz);
    dx = (double)sx / sqrt(1.0 + (double)sx * sx + (double)sy * sy + (double)sz * sz);
  };
  for (long long s = 0; s < a.steps; ++s) {
    const double t = a.t0 + (double)s * a.dt;
    double d1, d2, d3, d4;
    R a1, b1, c1, a2, b2, c2, a3, b3, c3, a4, b4, c4;
    stage(x, t, ux, uy, uz, d1, a1, b1, c1);
    stage(x + 0.5 * a.dt * d1, t + 0.5 * a.dt, ux + R(0.5) * h * a1, uy + R(0.5) * h * b1,
          uz + R(0.5) * h * c1, d2, a2, b2, c2);
    stage(x + 0.5 * a.dt * d2, t + 0.5 * a.dt, ux + R(0.5) * h * a2, uy + R(0.5) * h * b2,
          uz + R(0.5) * h * c2, d3, a3, b3, c3);
    stage(x + a.dt * d3, t + a.dt, ux + h * a3, uy + h * b3, uz + h * c3, d4, a4, b4, c4);
    x += a.dt / 6.0 * (d1 + 2.0 * d2 + 2.0 * d3 + d4);
    ux += h / R(6) * (a1 + R(2) * a2 + R(2) * a3 + a4);
    uy += h / R(6) * (b1 + R(2) * b2 + R(2) * b3 + b4);
    uz += h / R(6) * (c1 + R(2) * c2 + R(2) * c3 + c4);
  }
  a.x[i] = x;
  a.ux[i] = ux;
  a.uy[i] = uy;
  a.uz[i] = uz;
}

// ---------------------------------------------------------------- self-check
// Floats with bit patterns first .. first + count - 1 (those >= 1): count the
// results of sqrt_rn_ge1 and rcp_rn_ge1 (below 2^126) that differ from the
// correctly rounded sqrtf and 1.0f / x.
__global__ void k_check_rounding(unsigned first, unsigned count, unsigned long long* bad) {
  unsigned long long mine = 0;
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long k = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; k < count; k += stride) {
    const float x = __uint_as_float(first + (unsigned)k);
    if (!(x >= 1.0f) || !(x <= 3.4028235e38f)) continue;
    mine += __float_as_uint(sqrt_rn_ge1(x)) != __float_as_uint(sqrtf(x));
    if (x < 0x1p126f) mine += __float_as_uint(rcp_rn_ge1(x)) != __float_as_uint(1.0f / x);
  }
  if (mine) atomicAdd(bad, mine);
}

// ---------------------------------------------------------------- batched runs
// One slot per resident run.  Everything a step needs is derived from the
// run's device step counter n: sort due iff n > 0 and n % K == 0, particle
// buffer parity (n / K) & 1 for the push (the sort at step n reads parity
// (n / K - 1) & 1), field and current parity n & 1, laser time from n.  A
// captured sequence of batched launches can therefore be replayed while
// runs join and leave: only the slot table and the work ranges change.
template <typename R>
struct SlotDev {
  PushArgs<R> push[2][2];   // [particle parity][field parity]
  FieldArgs<R> field[2];    // [field parity]; tick = 0 (the field pass advances the counter itself)
  SortArgs<R> sort[2];      // [source particle parity]
  int* cnt[2];
  int* cur[2];
  long long* count;         // [parity][species]
  long long* step;          // the run's device step counter
  int* done;                // field chunks of the current step finished (zero between steps)
  long long target;         // the run stops once *step reaches target
  int sort_interval;
  int nx;
};

constexpr int kMaxSlots = 1024;
// ints between two slots' done counters: one 128-byte line each, so that the
// counting atomics of different runs do not queue on one line
constexpr int kDoneStride = 32;

// A value the whole wave shares, moved to scalar registers.
__device__ __forceinline__ long long uniform(long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(v & 0xffffffffll));
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// Work ranges of the slots, copied to LDS once per work-group; slot(b) is
// the slot whose range [start[s], start[s + 1]) holds work item b.
struct SlotRanges {
  int* st;  // LDS, n + 1 entries
  int n;
  // b is block-uniform, so is the result: readfirstlane lets the compiler
  // keep the slot (and every argument loaded through it) in scalar registers
  __device__ __forceinline__ int slot(int b) const {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
      const int m = (lo + hi) >> 1;
      if (st[m] <= b)
        lo = m;
      else
        hi = m;
    }
    return __builtin_amdgcn_readfirstlane(lo);
  }
  __device__ __forceinline__ int first(int sl) const { return __builtin_amdgcn_readfirstlane(st[sl]); }
  __device__ __forceinline__ int total() const { return __builtin_amdgcn_readfirstlane(st[n]); }
};

__device__ __forceinline__ SlotRanges load_ranges(const int* start, int n, int* lds) {
  for (int i = threadIdx.x; i <= n; i += blockDim.x) lds[i] = start[i];
  __syncthreads();
  return SlotRanges{lds, n};
}

// Batched push and field launches run one work-group per work item: the host
// sets their grids to the resident total whenever the slot table changes (a
// grid-stride loop here would keep more values live and cost occupancy).
template <typename R>
__global__ PIC_PUSH_BOUNDS void k_push_batch(const SlotDev<R>* __restrict__ slots, const int* __restrict__ start, int n) {
  __shared__ unsigned long long lds[kLdsSlots];
  // the slot table and the deposit window share the LDS: every wave reads
  // the table before the barrier below, the window is cleared after it
  static_assert((kMaxSlots + 1) * sizeof(int) <= sizeof(lds), "slot ranges must fit the window");
  const SlotRanges sr = load_ranges(start, n, reinterpret_cast<int*>(lds));
  const int b = (int)blockIdx.x;
  if (b >= sr.total()) return;  // block-uniform, as are the returns below
  const int sl = sr.slot(b);
  const int tile = b - sr.first(sl);
  __syncthreads();
  const SlotDev<R>& S = slots[sl];
  const long long st = uniform(*S.step);
  if (st >= S.target) return;
  const int pp = (int)((st / S.sort_interval) & 1), fp = (int)(st & 1);
  push_one_tile<R, kBatchPPT, kBatchDepth>(S.push[pp][fp], tile, lds);
}

// The field pass also ends the step: the last of a run's chunks to finish
// advances the run's step counter (every chunk of the run has read the
// counter before it counts itself done).
template <typename R>
__global__ __launch_bounds__(kFieldChunk) void k_field_batch(const SlotDev<R>* __restrict__ slots,
                                                            const int* __restrict__ start, int n) {
  __shared__ int rng[kMaxSlots + 1];
  __shared__ R sm[field_lds_elems<kFieldChunk>()];
  const SlotRanges sr = load_ranges(start, n, rng);
  const int b = (int)blockIdx.x;
  if (b >= sr.total()) return;
  const int sl = sr.slot(b);
  const SlotDev<R>& S = slots[sl];
  const long long st = uniform(*S.step);
  if (st >= S.target) return;
  field_chunk<R, kFieldChunk>(S.field[st & 1], b - sr.first(sl), 0, sm);
  // relaxed: a block's read of the counter has returned (its value chose the
  // buffers) before the block counts itself; acquire/release ordering here
  // would write back and invalidate the L2 once per work-group
  if (threadIdx.x == 0) {
    const int chunks = sr.first(sl + 1) - sr.first(sl);
    if (__hip_atomic_fetch_add(S.done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == chunks - 1) {
      __hip_atomic_store(S.done, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *S.step = st + 1;
    }
  }
}

template <typename R>
__device__ __forceinline__ bool sort_due(const SlotDev<R>& S, int* q) {
  const long long st = uniform(*S.step);
  if (st >= S.target || st <= 0 || st % S.sort_interval) return false;
  *q = (int)((st / S.sort_interval - 1) & 1);
  return true;
}

template <typename R>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist_batch(const SlotDev<R>* __restrict__ slots,
                                                                 const int* __restrict__ start, int n) {
  __shared__ int rng[kMaxSlots + 1];
  const SlotRanges sr = load_ranges(start, n, rng);
  for (int b = (int)blockIdx.x; b < sr.total(); b += (int)gridDim.x) {
    const int sl = sr.slot(b);
    int q;
    if (!sort_due(slots[sl], &q)) continue;
    sort_hist_block<R>(slots[sl].sort[q], b - sr.first(sl));
  }
}

template <typename R>
__global__ __launch_bounds__(1024) void k_sort_scan_batch(const SlotDev<R>* slots, int n) {
  for (int w = (int)blockIdx.x; w < 2 * n; w += (int)gridDim.x) {
    const int sl = w >> 1, sp = w & 1;
    const SlotDev<R>& S = slots[sl];
    int q;
    if (!sort_due(S, &q)) continue;
    __syncthreads();
    sort_scan_species(S.cnt[sp], S.cur[sp], S.count + 2 * (q ^ 1) + sp, S.nx);
  }
}

template <typename R>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter_batch(const SlotDev<R>* __restrict__ slots,
                                                                    const int* __restrict__ start, int n) {
  __shared__ int rng[kMaxSlots + 1];
  const SlotRanges sr = load_ranges(start, n, rng);
  for (int b = (int)blockIdx.x; b < sr.total(); b += (int)gridDim.x) {
    const int sl = sr.slot(b);
    int q;
    if (!sort_due(slots[sl], &q)) continue;
    sort_scatter_block<R>(slots[sl].sort[q], b - sr.first(sl));
  }
}

// ---------------------------------------------------------------- persistent batched steps
// Grid-wide barrier for a launch whose work-groups are all resident at once
// (the host sizes the grid from the kernel's occupancy).  Arrivals count in
// kBarGroups group words and then in one top word, so that no word takes
// more than about G / kBarGroups same-address atomics; the last arrival
// bumps the generation word that the others poll.  A wait longer than
// `ticks` of the 100 MHz constant clock (one second in use) sets *err, and
// once *err is set every wait ends at once: a launch always finishes, and
// the host reports the error.  Words sit 128 bytes apart: [0] generation,
// [32] top, [64 + 32 g] group g.
constexpr int kBarGroups = 16;
constexpr int kBarWords = 32 * (2 + kBarGroups);
constexpr unsigned long long kBarTicks = 100000000ull;  // one second

__device__ __forceinline__ void grid_sync(unsigned* w, int* err, unsigned long long ticks) {
  // every wave's loads and stores complete, then one agent-scope release per
  // work-group (an L2 write-back), relaxed counting and polling, and one
  // acquire after the wait (polling with acquire loads would invalidate the
  // caches on every poll, under the work-groups still running)
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned G = gridDim.x, g = blockIdx.x % kBarGroups;
    const unsigned in_g = (G - 1 - g) / kBarGroups + 1;  // blocks b < G with b % kBarGroups == g
    const unsigned groups = G < (unsigned)kBarGroups ? G : (unsigned)kBarGroups;
    unsigned* gen = w;
    const unsigned cur = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool last = false;
    unsigned* gw = w + 64 + 32 * g;
    // the last arrival of a group and the last overall pass the others'
    // releases on (acquire, then release, through a fence each)
    if (__hip_atomic_fetch_add(gw, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == in_g - 1) {
      __hip_atomic_store(gw, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      if (__hip_atomic_fetch_add(w + 32, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == groups - 1) {
        __hip_atomic_store(w + 32, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = true;
      }
    }
    if (!last) {
      const unsigned long long t0 = wall_clock64();
      while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == cur) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        if (wall_clock64() - t0 > ticks) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Slots a persistent launch serves (its range tables live in LDS beside the
// push window, and more of them would cost the push a work-group per CU).
constexpr int kPersistSlots = 128;

// `steps` batched steps in one launch: every work-group takes push tiles of
// all resident runs in turn, then field chunks of kThreads nodes, with a
// grid-wide barrier after each pass.  A run's step counter stays put during
// the launch (every pass computes its step as counter + k) and advances once
// at the end, by the number of steps the run had left, at most `steps`.
template <typename R>
__global__ __launch_bounds__(kThreads, PIC_STEPS_MIN_WAVES) void k_steps_batch(const SlotDev<R>* __restrict__ slots,
                                              const int* __restrict__ push_start,
                                              const int* __restrict__ field_start, int n, int steps,
                                              unsigned* bar, int* err, unsigned long long ticks) {
  __shared__ unsigned long long lds[kLdsSlots];
  __shared__ int rp[kPersistSlots + 1], rf[kPersistSlots + 1];
  static_assert(field_lds_elems<kThreads>() * sizeof(double) <= sizeof(lds), "field chunk must fit the window");
  for (int i = threadIdx.x; i <= n; i += blockDim.x) {
    rp[i] = push_start[i];
    rf[i] = field_start[i];
  }
  __syncthreads();
  const SlotRanges P{rp, n}, F{rf, n};
  const int G = (int)gridDim.x;
  for (int k = 0; k < steps; ++k) {
    for (int b = (int)blockIdx.x; b < P.total(); b += G) {
      const int sl = P.slot(b);
      const SlotDev<R>& S = slots[sl];
      const long long st = uniform(*S.step) + k;
      if (st >= S.target) continue;
      const int pp = (int)((st / S.sort_interval) & 1), fp = (int)(st & 1);
      __syncthreads();  // the block's previous tile is out of the window
      push_one_tile<R, kBatchPPT, kBatchDepth>(S.push[pp][fp], b - P.first(sl), lds);
    }
    grid_sync(bar, err, ticks);
    for (int b = (int)blockIdx.x; b < F.total(); b += G) {
      const int sl = F.slot(b);
      const SlotDev<R>& S = slots[sl];
      const long long st = uniform(*S.step) + k;
      if (st >= S.target) continue;
      __syncthreads();
      field_chunk<R, kThreads>(S.field[st & 1], b - F.first(sl), k, reinterpret_cast<R*>(lds));
    }
    grid_sync(bar, err, ticks);
  }
  // every work-group has read the counters before the last barrier
  if (blockIdx.x == 0) {
    for (int sl = threadIdx.x; sl < n; sl += blockDim.x) {
      long long* p = slots[sl].step;
      const long long v = *p, t = slots[sl].target;
      if (v < t) *p = v + steps < t ? v + steps : t;
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

// Kinetic energy (FP64) and integer charge of the particles.  Each block
// walks sort-sized tiles (blocks of a species stride over its tiles in a
// fixed order); the charge of a tile is gathered in an LDS window and added
// to HBM with one atomic per node.
template <typename R>
__global__ __launch_bounds__(kDiagThreads) void k_diag_particles(DiagArgs<R> p) {
  static_assert(kDiagThreads == kSortThreads, "diag tiles reuse the sort tiling");
  __shared__ double sh[kDiagThreads / 64];
  __shared__ long long sa[kDiagThreads / 64];
  __shared__ unsigned long long rw[kSortWin + 1];
  __shared__ int sm[8];
  const int s = blockIdx.x < kDiagPartBlocks ? 0 : 1;
  const int b = blockIdx.x - s * kDiagPartBlocks;
  const long long n = p.count[s];
  const SpeciesDev<R> sp = p.sp[s];
  const int lane = threadIdx.x & 63;
  double ke = 0.0;
  long long alive = 0;
  for (long long base = (long long)b * kSortTile; base < n;
       base += (long long)kDiagPartBlocks * kSortTile) {
    int cl[kSortPPT];
#pragma unroll
    for (int k = 0; k < kSortPPT; ++k) {
      const long long i = base + k * kSortThreads + threadIdx.x;
      cl[k] = i < n ? sp.cell[i] : kDead;
    }
    int lo, hi;
    tile_range(cl, lo, hi, sm);
    if (lo > hi) continue;  // block-uniform
    const int W = hi - lo + 2;  // nodes lo .. hi + 1
    const bool win = W <= kSortWin + 1;
    if (win) {
      for (int e = threadIdx.x; e < W; e += kSortThreads) rw[e] = 0ull;
      __syncthreads();
    }
#pragma unroll 4
    for (int k = 0; k < kSortPPT; ++k) {
      const long long i = base + k * kSortThreads + threadIdx.x;
      const int c = cl[k];
      const bool valid = c != kDead;
      long long r0 = 0, r1 = 0;
      if (valid) {
        const double ux = sp.ux[i], uy = sp.uy[i], uz = sp.uz[i];
        const double g = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
        ke += (double)sp.w[i] * p.mass[s] * (g - 1.0);
        const int q = (int)(sp.off[i] * R(kTwo24));
        const int qw = p.Z[s] * (int)rint(sp.w[i] * p.sw);
        r0 = (long long)qw * (kTwo24 - q);
        r1 = (long long)qw * q;
        alive += 1;
      }
      // wave-aggregate equal cells, then one add per distinct cell
      unsigned long long active = __ballot(valid);
      while (active) {
        const int leader = __ffsll((long long)active) - 1;
        const int lc = __shfl(c, leader);
        const bool mine = valid && c == lc && ((active >> lane) & 1ull);
        const long long a0 = wave_sum(mine ? r0 : 0ll);
        const long long a1 = wave_sum(mine ? r1 : 0ll);
        if (lane == leader) {
          if (win) {
            atomicAdd(rw + (lc - lo), (unsigned long long)a0);
            atomicAdd(rw + (lc - lo) + 1, (unsigned long long)a1);
          } else {
            atomicAdd((unsigned long long*)p.rho + lc + 1, (unsigned long long)a0);
            atomicAdd((unsigned long long*)p.rho + lc + 2, (unsigned long long)a1);
          }
        }
        active &= ~__ballot(mine);
      }
    }
    if (win) {
      __syncthreads();
      for (int e = threadIdx.x; e < W; e += kSortThreads)
        if (rw[e]) atomicAdd((unsigned long long*)p.rho + lo + e + 1, rw[e]);
      __syncthreads();
    }
  }
  const double t = block_sum(ke, sh);
  const long long na = wave_sum((long long)alive);
  if (lane == 0) sa[threadIdx.x >> 6] = na;
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
    const NodeF<R> nv = p.f.N[i];
    const double ey = nv.ey, ez = nv.ez;
    ue += wn * (ey * ey + ez * ez);
    if (i >= 1) {  // half-node h = i covers cell i-1
      const HalfF<R> hv = p.f.H[i];
      const double ex = hv.ex, by = hv.by, bz = hv.bz;
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

// fixed-order parallel reduction: thread t sums entries t, t + 256, ...,
// then a fixed tree over threads
__device__ __forceinline__ double fixed_sum(const double* x, int n, int stride, int off,
                                            double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += x[(size_t)i * stride + off];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_diag_final(const double* part, const long long* ipart,
                                                    const double* acc, int tiles,
                                                    DiagOutDev* out) {
  __shared__ double sh[256];
  const int base = 2 * kDiagPartBlocks;
  DiagOutDev o{};
  o.K_e = fixed_sum(part, kDiagPartBlocks, 1, 0, sh);
  o.K_i = fixed_sum(part + kDiagPartBlocks, kDiagPartBlocks, 1, 0, sh);
  o.U_Ex = fixed_sum(part + base, kDiagFieldBlocks, 1, 0, sh);
  o.U_Et = fixed_sum(part + base + kDiagFieldBlocks, kDiagFieldBlocks, 1, 0, sh);
  o.U_B = fixed_sum(part + base + 2 * kDiagFieldBlocks, kDiagFieldBlocks, 1, 0, sh);
  o.E_rad = fixed_sum(acc, tiles, 4, 0, sh);
  o.E_esc = fixed_sum(acc, tiles, 4, 1, sh) + fixed_sum(acc, tiles, 4, 2, sh);
  o.n_stiff = fixed_sum(acc, tiles, 4, 3, sh);
  if (threadIdx.x == 0) {
    for (int b = 0; b < kDiagPartBlocks; ++b) {
      o.alive0 += ipart[kDiagFieldBlocks + b];
      o.alive1 += ipart[kDiagFieldBlocks + kDiagPartBlocks + b];
    }
    for (int b = 0; b < kDiagFieldBlocks; ++b)
      o.gauss_int = ipart[b] > o.gauss_int ? ipart[b] : o.gauss_int;
    *out = o;
  }
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

// ---------------------------------------------------------------- friction coefficient
// The friction coefficient d of Eq. (damping) of every electron at the
// current step: d = eps gamma^2 [f_L^2 - (v.f_L)^2], f_L = -(E + v x B), with
// E^n, B^n gathered at x^n by the push's linear weights and v from the stored
// momentum; FP64 throughout.  Each electron adds its weight (FP64) to bin
// floor((log10 d - lo) / (hi - lo) bins), or to the under (d <= 0 or below
// lo) or over slot; a block's maximum of d and sums of w d and w go out with
// one atomic each.  out[bins + 0]: under, [+1]: over, [+2]: max d (bits: d >= 0
// orders as an integer), [+3]: sum of w d, [+4]: sum of w.
template <typename R>
__global__ __launch_bounds__(256) void k_friction(SpeciesDev<R> sp, FieldsDev<R> f,
                                                  const long long* count, double* out, int bins,
                                                  double lo, double hi, double eps) {
  __shared__ double s_max[256], s_sum[256], s_w[256];
  const long long n = *count;
  double dmax = 0.0, wd = 0.0, ws = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int c = sp.cell[i];
    if (c == kDead) continue;
    const double o = sp.off[i], on = 1.0 - o;
    const NodeF<R> n0 = f.N[c], n1 = f.N[c + 1];
    const double ey = on * (double)n0.ey + o * (double)n1.ey;
    const double ez = on * (double)n0.ez + o * (double)n1.ez;
    const double sx = o + 0.5;
    const int hb = sx >= 1.0;
    const double fh = hb ? sx - 1.0 : sx, fn = 1.0 - fh;
    const HalfF<R> h0 = f.H[c + hb], h1 = f.H[c + hb + 1];
    const double ex = fn * (double)h0.ex + fh * (double)h1.ex;
    const double by = fn * (double)h0.by + fh * (double)h1.by;
    const double bz = fn * (double)h0.bz + fh * (double)h1.bz;
    const double ux = sp.ux[i], uy = sp.uy[i], uz = sp.uz[i];
    const double g2 = 1.0 + ux * ux + uy * uy + uz * uz, g = sqrt(g2);
    const double vx = ux / g, vy = uy / g, vz = uz / g;
    // f_L = -(E + v x B), B = (0, by, bz)
    const double fx = -(ex + (vy * bz - vz * by));
    const double fy = -(ey - vx * bz);
    const double fz = -(ez + vx * by);
    const double vf = vx * fx + vy * fy + vz * fz;
    const double d = eps * g2 * ((fx * fx + fy * fy + fz * fz) - vf * vf);
    const double w = sp.w[i];
    const double l = d > 0.0 ? log10(d) : -INFINITY;
    long long b = l < lo ? -1 : (l >= hi ? bins : (long long)floor((l - lo) / (hi - lo) * bins));
    if (b >= bins) b = l >= hi ? bins : bins - 1;  // l just below hi
    atomicAdd(out + (b < 0 ? bins : (b >= bins ? bins + 1 : b)), w);
    if (d > dmax) dmax = d;
    wd += w * d;
    ws += w;
  }
  s_max[threadIdx.x] = dmax;
  s_sum[threadIdx.x] = wd;
  s_w[threadIdx.x] = ws;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      s_max[threadIdx.x] = fmax(s_max[threadIdx.x], s_max[threadIdx.x + k]);
      s_sum[threadIdx.x] += s_sum[threadIdx.x + k];
      s_w[threadIdx.x] += s_w[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(reinterpret_cast<unsigned long long*>(out + bins + 2),
              (unsigned long long)__double_as_longlong(s_max[0]));
    atomicAdd(out + bins + 3, s_sum[0]);
    atomicAdd(out + bins + 4, s_w[0]);
  }
}

}  // namespace pic
