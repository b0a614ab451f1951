// Device code of the 2D3V path (gfx950): the momentum step of the 1D3V
// kernels (Boris plus the RR step of Section 3) on a 2D Yee grid, periodic
// in y.  Section 4 notes that the 1D code's momentum space is already three
// dimensional, so a multi-dimensional code uses the same pusher; here it is
// the same device function, with B_x switched on.
//
// Kernels:
//   k_push2     gather -> Boris -> RR (electrons) -> 2D move -> fixed-point
//               Esirkepov deposit, one thread per particle over cell-sorted
//               tiles of 1,024.  A tile first stages the fields of its cells
//               in LDS and gathers from there; each lane adds the non-zero
//               terms of its particle's 3 x 3 stencil to one of several
//               private copies of an LDS box covering the tile's cells; the
//               box goes to HBM with one 64-bit atomic per node at the end.
//   k_field2    one Yee step (B half step, E step, B half step) per tile
//               with halos recomputed in LDS, boundary guards, Poynting
//               bookkeeping, the running integer charge implied by the
//               current, and the clearing of the next step's current.
//   k_field2m   the same step in column-marching form: a work-group owns a
//               strip of columns and the whole period (one thread per row)
//               and streams along x, reading each value once; used where
//               the period fits one work-group.
//   k_init2, k_diag2_*: quiet start and FP64 diagnostics.
// The cell sort reuses the 1D kernels (the y offset moves with the particle).
//
// Cell key of a particle: ix << ysh | iy (ysh = bits of ny rounded up to a
// power of two), so that (ix, iy) decode with a shift and a mask.  The
// counting sort orders particles by blocks of 8 x 8 cells (sort_key2), so
// that a push tile covers a compact patch of cells.  Grid
// arrays are y-fastest with stride ny: component at (column X, row j) is
// element X * ny + j.
#pragma once

#include "kernels.hpp"

namespace pic {

#ifndef PIC2D_PUSH_PPT
#define PIC2D_PUSH_PPT 4
#endif
#ifndef PIC2D_SORT_BLOCK
#define PIC2D_SORT_BLOCK 3
#endif
#ifndef PIC2D_LDS_SLOTS
#define PIC2D_LDS_SLOTS 3072
#endif

constexpr int k2SortBlock = PIC2D_SORT_BLOCK;  // log2 of the sort blocks' side in cells
constexpr int k2Q = 12;                   // fixed-point bits of a shape weight
constexpr int k2One = 1 << k2Q;
constexpr int k2PPT = PIC2D_PUSH_PPT;     // particles per thread per tile
constexpr int k2Tile = kThreads * k2PPT;
constexpr int k2Slots = PIC2D_LDS_SLOTS;  // 64-bit LDS accumulators per work-group
#ifndef PIC2D_MAX_COPIES
#define PIC2D_MAX_COPIES 8
#endif
constexpr int k2MaxCopies = PIC2D_MAX_COPIES;  // private LDS copies per current slot, at most

// staggered field pairs: (E_y, B_x) at (node, half-row), (E_x, B_y) at (half-node, row)
template <typename R>
struct alignas(2 * sizeof(R)) NH {
  R ey, bx;
};
template <typename R>
struct alignas(2 * sizeof(R)) HN {
  R ex, by;
};

template <typename R>
struct Fields2Dev {
  R* ez;       // [(nx + 1) ny]  node, row
  NH<R>* nh;   // [(nx + 1) ny]  node, half-row
  HN<R>* hn;   // [(nx + 2) ny]  half-node, row
  R* bz;       // [(nx + 2) ny]  half-node, half-row
};

template <typename R>
struct Push2Args {
  SpeciesDev<R> sp[2];          // with oy
  const long long* count;       // [2] particles per species as of the last sort
  int tiles0;                   // work-groups of species 0
  int ntiles;
  Fields2Dev<R> f;              // E^n, B^n
  unsigned long long* J[3];     // Jx [(nx + 2) ny], Jy, Jz [(nx + 3) ny] (node + 1)
  double* acc;                  // [tile][4] cumulative: E_rad, E_esc_e, E_esc_i, n_stiff
  int* flags;                   // [0]: non-finite seen
  int nx, ny, ysh;
  R cfl;                        // dt / dx = dt / dy
  R dt;
  R eps;
  R qh[2];
  int Z[2];
  double mass[2];
  int rr0;
  int comp;
  R sw;                         // 256 / w_ref
  int qw_ref[2];
};

template <typename R>
struct P2 {
  int c;
  R ox, oy, ux, uy, uz, w;
  float rx, ry, rz;
};

// loads of particle i (cell already known); past the end, particle n - 1
// is read instead and the cell says removed
template <typename R, bool COMP>
__device__ __forceinline__ P2<R> load2(const SpeciesDev<R>& sp, int i, int n, int c) {
  P2<R> d;
  const unsigned ui = (unsigned)(i < n ? i : n - 1);
  d.c = c;
  d.ox = ld(sp.off, ui);
  d.oy = ld(sp.oy, ui);
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

// E^n, B^n at a particle: bilinear weights of each component at its own
// staggered position
template <typename R>
__device__ __forceinline__ void gather2(const Fields2Dev<R>& f, int ny, int ix, int iy, R ox, R oy,
                                        R& ex, R& ey, R& ez, R& bx, R& by, R& bz) {
  const unsigned j0 = (unsigned)iy, j1 = iy + 1 == ny ? 0u : (unsigned)(iy + 1);
  const bool gb = oy >= R(0.5);                 // half-rows g0, g0 + 1 around the particle
  const unsigned g0 = gb ? j0 : (iy == 0 ? (unsigned)(ny - 1) : j0 - 1), g1 = gb ? j1 : j0;
  const R fy = gb ? oy - R(0.5) : oy + R(0.5);
  const bool hb = ox >= R(0.5);                 // half-nodes h0, h0 + 1
  const R fx = hb ? ox - R(0.5) : ox + R(0.5);
  const unsigned n0 = (unsigned)ix * (unsigned)ny, n1 = n0 + (unsigned)ny;
  const unsigned q0 = n0 + (hb ? (unsigned)ny : 0u), q1 = q0 + (unsigned)ny;
  const R wx0 = R(1) - ox, wy0 = R(1) - oy, vx0 = R(1) - fx, vy0 = R(1) - fy;
  {
    const R a = ld(f.ez, n0 + j0), b = ld(f.ez, n0 + j1), c = ld(f.ez, n1 + j0), d = ld(f.ez, n1 + j1);
    ez = wx0 * (wy0 * a + oy * b) + ox * (wy0 * c + oy * d);
  }
  {
    const NH<R> a = ld(f.nh, n0 + g0), b = ld(f.nh, n0 + g1), c = ld(f.nh, n1 + g0),
                d = ld(f.nh, n1 + g1);
    ey = wx0 * (vy0 * a.ey + fy * b.ey) + ox * (vy0 * c.ey + fy * d.ey);
    bx = wx0 * (vy0 * a.bx + fy * b.bx) + ox * (vy0 * c.bx + fy * d.bx);
  }
  {
    const HN<R> a = ld(f.hn, q0 + j0), b = ld(f.hn, q0 + j1), c = ld(f.hn, q1 + j0),
                d = ld(f.hn, q1 + j1);
    ex = vx0 * (wy0 * a.ex + oy * b.ex) + fx * (wy0 * c.ex + oy * d.ex);
    by = vx0 * (wy0 * a.by + oy * b.by) + fx * (wy0 * c.by + oy * d.by);
  }
  {
    const R a = ld(f.bz, q0 + g0), b = ld(f.bz, q0 + g1), c = ld(f.bz, q1 + g0), d = ld(f.bz, q1 + g1);
    bz = vx0 * (vy0 * a + fy * b) + fx * (vy0 * c + fy * d);
  }
}

// Position update of the 2D contract: the 1D arithmetic in x and in y.
template <typename R>
__device__ __forceinline__ void contract_move2(R ux, R uy, R uz, R ox, R oy, R cfl, R& g, R& vz,
                                               R& ox1, R& oy1, R& sx, R& sy) {
#pragma clang fp contract(off)
  g = sqrt_rn_ge1(((R(1) + ux * ux) + uy * uy) + uz * uz);
  const R ig = rcp_rn_ge1(g);
  const R vx = ux * ig, vy = uy * ig;
  vz = uz * ig;
  R s = ox + vx * cfl;
  R fl = floor(s);
  ox1 = s - fl;
  if (ox1 >= R(1)) {
    ox1 = R(0);
    fl += R(1);
  }
  sx = fl;
  s = oy + vy * cfl;
  fl = floor(s);
  oy1 = s - fl;
  if (oy1 >= R(1)) {
    oy1 = R(0);
    fl += R(1);
  }
  sy = fl;
}

// 12-bit weights of one direction on the three nodes base .. base + 2,
// base = min(old cell, new cell): the old cell sits at base + d0, the new
// one at base + d1 (d0, d1 in {0, 1})
template <typename R>
__device__ __forceinline__ void shapes2(R o, R o1, int sh, int (&S0)[3], int (&S1)[3]) {
  const int q0 = (int)(o * R(k2One)), q1 = (int)(o1 * R(k2One));
  const bool d0 = sh < 0, d1 = sh > 0;
  S0[0] = d0 ? 0 : k2One - q0;
  S0[1] = d0 ? k2One - q0 : q0;
  S0[2] = d0 ? q0 : 0;
  S1[0] = d1 ? 0 : k2One - q1;
  S1[1] = d1 ? k2One - q1 : q1;
  S1[2] = d1 ? q1 : 0;
}

// LDS current box of one tile: BX columns from xmn (Jx: half-node
// h = xmn + c; Jy, Jz: node index xmn + c, i.e. node xmn - 1 + c) and BY
// rows from jbase (mod ny); slot (comp, r, c) = (comp BY + r) BX + c.  NC
// private copies of the whole box, CS words apart (CS odd, so that the same
// slot of different copies falls in different banks); lane & (NC - 1)
// picks the copy, so that lanes of a wave in one cell add to different words
struct Box2 {
  unsigned long long* lds;
  int xmn, jbase, BX, BY, NC, CS;
  int copy;                  // offset of this lane's copy
  bool use;
};

// The fixed-point Esirkepov current of one move (the 2D deposition
// contract), added term by term to the box (or to HBM when the tile has no
// box).  With base = min(old, new) cell in each direction and 3-node weights
// S0 (old), S1 (new): C[a] = sum_{a' <= a} (S0 - S1)[a'], Sig = S0 + S1,
//   Jx(face base + a + 1/2, row b) += qw C_x[a] Sig_y[b]      a < 2, b < 3
//   Jy(node a, half-row base + b + 1/2) += qw Sig_x[a] C_y[b]  a < 3, b < 2
//   Jz(node a, row b) += qw rint(v_z 2^12) ((S0_x S0_y + S1_x S1_y)[a, b] >> 12).
// Terms that vanish for a move without a cell change in x (face 1, node 2)
// or y (row 2, half-row 1) are not added.  Every term is below 2^25, so the
// 24-bit multiplies are exact.  Terms of particles with the reference weight
// go to the box as multiples of it.
struct Terms2 {
  int X0[3], X1[3], Y0[3], Y1[3], Cx[2], Cy[2], vz12;
  bool mx, my;
  __device__ __forceinline__ int jx(int i, int j) const { return __mul24(Cx[i], Y0[j] + Y1[j]); }
  __device__ __forceinline__ int jy(int i, int j) const { return __mul24(X0[i] + X1[i], Cy[j]); }
  __device__ __forceinline__ int jz(int i, int j) const {
    return __mul24(vz12, (__mul24(X0[i], Y0[j]) + __mul24(X1[i], Y1[j])) >> k2Q);
  }
};

template <typename R>
__device__ __forceinline__ Terms2 terms2(R ox, R oy, R ox1, R oy1, int sx, int sy, R vz) {
  Terms2 t;
  shapes2<R>(ox, ox1, sx, t.X0, t.X1);
  shapes2<R>(oy, oy1, sy, t.Y0, t.Y1);
  t.Cx[0] = t.X0[0] - t.X1[0];
  t.Cx[1] = t.Cx[0] + (t.X0[1] - t.X1[1]);
  t.Cy[0] = t.Y0[0] - t.Y1[0];
  t.Cy[1] = t.Cy[0] + (t.Y0[1] - t.Y1[1]);
  t.vz12 = (int)rint(vz * R(k2One));
  t.mx = sx != 0;
  t.my = sy != 0;
  return t;
}

// add the terms through `put(comp, column offset, row b, value)` (columns
// and rows counted from the stencil base)
template <typename Put>
__device__ __forceinline__ void add_terms2(const Terms2& t, Put&& put) {
  put(0, 0, 0, t.jx(0, 0));
  put(0, 0, 1, t.jx(0, 1));
  put(1, 0, 0, t.jy(0, 0));
  put(1, 1, 0, t.jy(1, 0));
  put(2, 0, 0, t.jz(0, 0));
  put(2, 1, 0, t.jz(1, 0));
  put(2, 0, 1, t.jz(0, 1));
  put(2, 1, 1, t.jz(1, 1));
  if (t.mx) {
    put(0, 1, 0, t.jx(1, 0));
    put(0, 1, 1, t.jx(1, 1));
    put(1, 2, 0, t.jy(2, 0));
    put(2, 2, 0, t.jz(2, 0));
    put(2, 2, 1, t.jz(2, 1));
  }
  if (t.my) {
    put(0, 0, 2, t.jx(0, 2));
    put(1, 0, 1, t.jy(0, 1));
    put(1, 1, 1, t.jy(1, 1));
    put(2, 0, 2, t.jz(0, 2));
    put(2, 1, 2, t.jz(1, 2));
    if (t.mx) {
      put(0, 1, 2, t.jx(1, 2));
      put(1, 2, 1, t.jy(2, 1));
      put(2, 2, 2, t.jz(2, 2));
    }
  }
}

template <typename R>
__device__ __forceinline__ void deposit2(const Push2Args<R>& a, const Box2& bx, int ix, int iy, R ox,
                                         R oy, R ox1, R oy1, int sx, int sy, R vz, int qw, int qw_ref) {
  const Terms2 t = terms2<R>(ox, oy, ox1, oy1, sx, sy, vz);
  const int ny = a.ny;
  const int bxn = min(ix, ix + sx) + 1;  // column index of node base (guard offset 1)
  const int by0 = min(iy, iy + sy);      // base row, -1 .. ny - 1 before wrapping
  if (bx.use && qw == qw_ref) {
    // slot of (comp, row b, column 0) in this lane's copy: row offsets per
    // lane, component offsets uniform, columns immediate
    int ro[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      int r = by0 + b - bx.jbase;
      r += r < 0 ? ny : 0;
      r -= r >= ny ? ny : 0;
      ro[b] = r * bx.BX + (bxn - bx.xmn) + bx.copy;
    }
    const int P = bx.BY * bx.BX;
    add_terms2(t, [&](int comp, int ca, int b, int v) {
      atomicAdd(bx.lds + (ro[b] + comp * P) + ca, (unsigned long long)(long long)v);
    });
  } else {
    int rg[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      int r = by0 + b;
      r += r < 0 ? ny : 0;
      r -= r >= ny ? ny : 0;
      rg[b] = r;
    }
    const long long q = qw;
    add_terms2(t, [&](int comp, int ca, int b, int v) {
      atomicAdd(a.J[comp] + (size_t)(bxn + ca) * ny + rg[b], (unsigned long long)(q * v));
    });
  }
}

// Fields of one tile staged in LDS: columns x0 .. x0 + SX - 1 (node and
// half-node columns alike), rows of the tile's arc from one below to one
// above, SY of them, row fastest per class array.  A particle in cell
// (ix, iy) reads columns ix - x0 .. + 2 and rows iy - 1 .. iy + 1, which are
// local rows r0 .. r0 + 2 with r0 = (iy - 1 - row0) mod ny.
#ifndef PIC2D_FIELD_STAGE
#define PIC2D_FIELD_STAGE 384
#endif
constexpr int k2Stage = PIC2D_FIELD_STAGE;  // staged (column, row) cells per tile, at most

template <typename R>
struct Stage2 {
  const R* ez;
  const NH<R>* nh;
  const HN<R>* hn;
  const R* bz;
  int x0, row0, SY;
  bool use;
};

template <typename R>
__device__ __forceinline__ void gather2_lds(const Stage2<R>& g, int ny, int ix, int iy, R ox, R oy,
                                            R& ex, R& ey, R& ez, R& bx, R& by, R& bz) {
  int r0 = iy - 1 - g.row0;
  r0 += r0 < 0 ? ny : 0;
  r0 -= r0 >= ny ? ny : 0;
  const int gb = oy >= R(0.5), hb = ox >= R(0.5);
  const R fy = gb ? oy - R(0.5) : oy + R(0.5);
  const R fx = hb ? ox - R(0.5) : ox + R(0.5);
  const int n0 = (ix - g.x0) * g.SY, n1 = n0 + g.SY;
  const int q0 = n0 + (hb ? g.SY : 0), q1 = q0 + g.SY;
  const int rj = r0 + 1, rg = r0 + gb;  // first row, first half-row
  const R wx0 = R(1) - ox, wy0 = R(1) - oy, vx0 = R(1) - fx, vy0 = R(1) - fy;
  ez = wx0 * (wy0 * g.ez[n0 + rj] + oy * g.ez[n0 + rj + 1]) +
       ox * (wy0 * g.ez[n1 + rj] + oy * g.ez[n1 + rj + 1]);
  {
    const NH<R> a = g.nh[n0 + rg], b = g.nh[n0 + rg + 1], c = g.nh[n1 + rg], d = g.nh[n1 + rg + 1];
    ey = wx0 * (vy0 * a.ey + fy * b.ey) + ox * (vy0 * c.ey + fy * d.ey);
    bx = wx0 * (vy0 * a.bx + fy * b.bx) + ox * (vy0 * c.bx + fy * d.bx);
  }
  {
    const HN<R> a = g.hn[q0 + rj], b = g.hn[q0 + rj + 1], c = g.hn[q1 + rj], d = g.hn[q1 + rj + 1];
    ex = vx0 * (wy0 * a.ex + oy * b.ex) + fx * (wy0 * c.ex + oy * d.ex);
    by = vx0 * (wy0 * a.by + oy * b.by) + fx * (wy0 * c.by + oy * d.by);
  }
  bz = vx0 * (vy0 * g.bz[q0 + rg] + fy * g.bz[q0 + rg + 1]) +
       fx * (vy0 * g.bz[q1 + rg] + fy * g.bz[q1 + rg + 1]);
}

struct Acc2 {
  float rad, esc, stiff;
};

// One particle: gather, Boris with RR, 2D move, stores; fills the deposit
// terms (zero and dep = false for removed particles).
template <typename R, bool RR, bool COMP>
__device__ __forceinline__ void push2_particle(const Push2Args<R>& a, const SpeciesDev<R>& sp, int s,
                                               unsigned ui, const P2<R>& pd, const Box2& box,
                                               const Stage2<R>& stg, Acc2& acc) {
  if (pd.c == kDead) return;
  const int ymask = (1 << a.ysh) - 1;
  const int ix = pd.c >> a.ysh, iy = pd.c & ymask;
  R ex, ey, ez, bx, by, bz;
  if (stg.use)
    gather2_lds<R>(stg, a.ny, ix, iy, pd.ox, pd.oy, ex, ey, ez, bx, by, bz);
  else
    gather2<R>(a.f, a.ny, ix, iy, pd.ox, pd.oy, ex, ey, ez, bx, by, bz);
  float rx = pd.rx, ry = pd.ry, rz = pd.rz;
  MomentumOut<R> mo;
  momentum_step<R, RR, COMP, false, true>(pd.ux, pd.uy, pd.uz, ex, ey, ez, by, bz, a.qh[s],
                                          a.eps * a.dt, FieldRates<R>{}, rx, ry, rz, acc.stiff, mo,
                                          bx);
  R g, vz, ox1, oy1, shx, shy;
  contract_move2<R>(mo.nx, mo.ny, mo.nz, pd.ox, pd.oy, a.cfl, g, vz, ox1, oy1, shx, shy);
  if (!(fabs(shx) < R(4)) || !(fabs(shy) < R(4)) || !(g < R(1e30))) {
    st(sp.cell, ui, kDead);
    atomicOr(a.flags, 1);
    return;
  }
  const int sx = (int)shx, sy = (int)shy;
  const int qw = a.Z[s] * (int)rint(pd.w * a.sw);
  deposit2<R>(a, box, ix, iy, pd.ox, pd.oy, ox1, oy1, sx, sy, vz, qw, a.qw_ref[s]);
  if (RR) {
    const R num = mo.ddx * (R(2) * mo.Lx + mo.ddx) + mo.ddy * (R(2) * mo.Ly + mo.ddy) +
                  mo.ddz * (R(2) * mo.Lz + mo.ddz);
    acc.rad -= (float)(pd.w * num * rcp(mo.gL + g));
  }
  const int ix1 = ix + sx;
  int iy1 = iy + sy;
  iy1 += iy1 < 0 ? a.ny : 0;
  iy1 -= iy1 >= a.ny ? a.ny : 0;
  if (ix1 < 0 || ix1 >= a.nx) {
    st(sp.cell, ui, kDead);
    acc.esc += (float)(pd.w * (R)a.mass[s] * (g - R(1)));
  } else {
    st(sp.cell, ui, (ix1 << a.ysh) | iy1);
    st(sp.off, ui, ox1);
    st(sp.oy, ui, oy1);
  }
  st(sp.ux, ui, mo.nx);
  st(sp.uy, ui, mo.ny);
  st(sp.uz, ui, mo.nz);
  if (COMP) {
    st(sp.rx, ui, rx);
    st(sp.ry, ui, ry);
    st(sp.rz, ui, rz);
  }
}

template <typename R, bool RR, bool COMP>
__device__ __forceinline__ void push2_tile(const Push2Args<R>& a, int s, int tile, int n, int base,
                                           unsigned long long* lds, R* fst) {
  __shared__ int s_red[4][kThreads / kLanes];
  __shared__ int s_jref;
  __shared__ double s_acc[3][kThreads / kLanes];
  const SpeciesDev<R> sp = a.sp[s];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int ny = a.ny, ymask = (1 << a.ysh) - 1;

  int cl[k2PPT];
#pragma unroll
  for (int k = 0; k < k2PPT; ++k) {
    const int i = base + k * kThreads + tid;
    cl[k] = i < n ? ld(sp.cell, (unsigned)i) : kDead;
  }
  // the tile's rows as an arc of the periodic y range around a reference
  // row (the first live particle of thread 0)
  if (tid == 0) {
    int jr = 0;
#pragma unroll
    for (int k = k2PPT - 1; k >= 0; --k)
      if (cl[k] != kDead) jr = cl[k] & ymask;
    s_jref = jr;
  }
  __syncthreads();
  const int jref = s_jref, half = ny >> 1;
  int xmn = INT_MAX, xmx = INT_MIN, dmn = INT_MAX, dmx = INT_MIN;
#pragma unroll
  for (int k = 0; k < k2PPT; ++k) {
    const int c = cl[k];
    if (c != kDead) {
      const int x = c >> a.ysh;
      int d = (c & ymask) - jref;
      d += d < -half ? ny : 0;
      d -= d >= ny - half ? ny : 0;
      xmn = min(xmn, x);
      xmx = max(xmx, x);
      dmn = min(dmn, d);
      dmx = max(dmx, d);
    }
  }
  xmn = wave_min_dpp(xmn);
  xmx = wave_max_dpp(xmx);
  dmn = wave_min_dpp(dmn);
  dmx = wave_max_dpp(dmx);
  if (lane == 0) {
    s_red[0][wid] = xmn;
    s_red[1][wid] = xmx;
    s_red[2][wid] = dmn;
    s_red[3][wid] = dmx;
  }
  __syncthreads();
  xmn = min(min(s_red[0][0], s_red[0][1]), min(s_red[0][2], s_red[0][3]));
  xmx = max(max(s_red[1][0], s_red[1][1]), max(s_red[1][2], s_red[1][3]));
  dmn = min(min(s_red[2][0], s_red[2][1]), min(s_red[2][2], s_red[2][3]));
  dmx = max(max(s_red[3][0], s_red[3][1]), max(s_red[3][2], s_red[3][3]));
  if (xmn > xmx) return;  // every particle of the tile was removed (block-uniform)

  // box: columns xmn - 1 .. xmx + 2, rows of the arc plus one below and two
  // above (or every row, the stencils wrapping onto it)
  Box2 bx;
  bx.xmn = xmn;
  bx.BX = xmx - xmn + 4;
  const int span = dmx - dmn + 4;
  if (span < ny) {
    bx.BY = span;
    int jb = jref + dmn - 1;
    jb += jb < 0 ? ny : 0;
    jb -= jb >= ny ? ny : 0;
    bx.jbase = jb;
  } else {
    bx.BY = ny;
    bx.jbase = 0;
  }
  const int slots = 3 * bx.BX * bx.BY;
  bx.CS = slots | 1;
  int nc = k2MaxCopies;
  while (nc > 1 && bx.CS * nc > k2Slots) nc >>= 1;
  bx.NC = nc;
  bx.use = bx.CS * nc <= k2Slots;
  bx.lds = lds;
  bx.copy = (lane & (nc - 1)) * bx.CS;
  if (bx.use)
    for (int e = tid; e < bx.CS * nc; e += kThreads) lds[e] = 0ull;

  // fields of the tile's cells: columns xmn .. xmx + 2, rows of the arc from
  // one below to one above (every row plus the two wrapped ones when the arc
  // covers the whole period)
  R* s_ez = reinterpret_cast<R*>(fst);
  R* s_bz = s_ez + k2Stage;
  NH<R>* s_nh = reinterpret_cast<NH<R>*>(s_bz + k2Stage);
  HN<R>* s_hn = reinterpret_cast<HN<R>*>(s_nh + k2Stage);
  Stage2<R> stg;
  stg.ez = s_ez;
  stg.nh = s_nh;
  stg.hn = s_hn;
  stg.bz = s_bz;
  stg.x0 = xmn;
  if (span < ny) {
    stg.SY = span - 1;
    stg.row0 = bx.jbase;
  } else {
    stg.SY = ny + 2;
    stg.row0 = ny - 1;
  }
  const int SX = xmx - xmn + 3;
  stg.use = SX * stg.SY <= k2Stage;
  if (stg.use) {
    for (int e = tid; e < SX * stg.SY; e += kThreads) {
      const int c = e / stg.SY, r = e - c * stg.SY;
      const int gx = xmn + c;
      int gy = stg.row0 + r;
      gy -= gy >= ny ? ny : 0;
      gy -= gy >= ny ? ny : 0;
      const size_t gi = (size_t)gx * ny + gy;
      const bool node = gx <= a.nx;  // node arrays end at column nx, half-node arrays at nx + 1
      s_ez[e] = node ? a.f.ez[gi] : R(0);
      s_nh[e] = node ? a.f.nh[gi] : NH<R>{R(0), R(0)};
      s_hn[e] = a.f.hn[gi];
      s_bz[e] = a.f.bz[gi];
    }
  }
  __syncthreads();

  Acc2 acc{0.f, 0.f, 0.f};
  P2<R> cur = load2<R, COMP>(sp, base + tid, n, cl[0]);
#pragma unroll 2
  for (int k = 0; k < k2PPT; ++k) {
    const int i = base + k * kThreads + tid;
    P2<R> nxt;
    if (k + 1 < k2PPT) nxt = load2<R, COMP>(sp, i + kThreads, n, cl[k + 1]);
    push2_particle<R, RR, COMP>(a, sp, s, (unsigned)i, cur, bx, stg, acc);
    if (k + 1 < k2PPT) cur = nxt;
  }

  const double r0 = wave_sum_dpp((double)acc.rad), r1 = wave_sum_dpp((double)acc.esc),
               r2 = wave_sum_dpp((double)acc.stiff);
  if (lane == 0) {
    s_acc[0][wid] = r0;
    s_acc[1][wid] = r1;
    s_acc[2][wid] = r2;
  }
  __syncthreads();
  if (bx.use) {
    const int P = bx.BX * bx.BY;
    const long long qw_ref = a.qw_ref[s];
    for (int e = tid; e < slots; e += kThreads) {
      long long v = 0;
      for (int k = 0; k < bx.NC; ++k) v += (long long)lds[k * bx.CS + e];
      if (v) {
        const int comp = e >= 2 * P ? 2 : (e >= P ? 1 : 0);
        const int rem = e - comp * P;
        const int r = rem / bx.BX, c = rem - r * bx.BX;
        int gy = bx.jbase + r;
        gy -= gy >= ny ? ny : 0;
        atomicAdd(a.J[comp] + (size_t)(xmn + c) * ny + gy, (unsigned long long)(v * qw_ref));
      }
    }
  }
  if (tid == 0) {
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int w = 0; w < kThreads / kLanes; ++w) {
      t0 += s_acc[0][w];
      t1 += s_acc[1][w];
      t2 += s_acc[2][w];
    }
    double* A = a.acc + 4 * (size_t)tile;
    unsafeAtomicAdd(A + 0, t0);
    unsafeAtomicAdd(A + 1 + s, t1);
    unsafeAtomicAdd(A + 3, t2);
  }
}

// one work-group per tile
#ifndef PIC2D_PUSH_MIN_WAVES
#define PIC2D_PUSH_MIN_WAVES 0
#endif
#if PIC2D_PUSH_MIN_WAVES > 0
#define PIC2D_PUSH_BOUNDS __launch_bounds__(kThreads, PIC2D_PUSH_MIN_WAVES)
#else
#define PIC2D_PUSH_BOUNDS __launch_bounds__(kThreads)
#endif

template <typename R>
__global__ PIC2D_PUSH_BOUNDS void k_push2(Push2Args<R> a) {
  __shared__ unsigned long long lds[k2Slots];
  __shared__ R fst[6 * k2Stage];  // staged fields: E_z, B_z, (E_y, B_x), (E_x, B_y)
  const int tile = (int)blockIdx.x;
  const int s = tile < a.tiles0 ? 0 : 1;
  const int tl = s ? tile - a.tiles0 : tile;
  const int n = (int)a.count[s];
  const int base = tl * k2Tile;
  if (base >= n) return;
  if (s == 0 && a.rr0) {
    if (a.comp)
      push2_tile<R, true, true>(a, s, tile, n, base, lds, fst);
    else
      push2_tile<R, true, false>(a, s, tile, n, base, lds, fst);
  } else {
    push2_tile<R, false, false>(a, s, tile, n, base, lds, fst);
  }
}

// Exclusive scan of the cell counts of a 2D grid (millions of keys): the
// chunks of both species in parallel, then each chunk adds the totals of the
// chunks before it; the last chunk writes the alive count.
__global__ __launch_bounds__(kScanThreads) void k_scan2_chunks(int* cnt0, int* cnt1, int* cur0,
                                                              int* cur1, int* tot, int nkeys,
                                                              int nchunks) {
  __shared__ int stage[kScanChunk];
  __shared__ int wsum[kScanThreads / kLanes];
  const int s = blockIdx.y, c = blockIdx.x;
  const int t = scan_chunk(s ? cnt1 : cnt0, s ? cur1 : cur0, c * kScanChunk, nkeys, 0, stage, wsum);
  if (threadIdx.x == 0) tot[s * nchunks + c] = t;
}

__global__ __launch_bounds__(kScanThreads) void k_scan2_offsets(int* cur0, int* cur1, const int* tot,
                                                               long long* new_count, int nkeys,
                                                               int nchunks) {
  __shared__ long long red[kScanThreads / kLanes];
  const int s = blockIdx.y, c = blockIdx.x, t = threadIdx.x;
  const int* T = tot + s * nchunks;
  long long v = 0;
  for (int k = t; k < c; k += kScanThreads) v += T[k];
  v = wave_sum(v);
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  long long off = 0;
  for (int w = 0; w < kScanThreads / kLanes; ++w) off += red[w];
  int* cur = s ? cur1 : cur0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int j = c * kScanChunk + k * kScanThreads + t;
    if (j < nkeys) cur[j] += (int)off;
  }
  if (c == nchunks - 1 && t == 0) new_count[s] = off + T[c];
}

// cell sort of 2D particles: the 1D passes, with the y offset moved too
template <typename R>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist2(SortArgs<R> p) {
  sort_hist_block<R, true>(p, (int)blockIdx.x);
}

template <typename R>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter2(SortArgs<R> p) {
  sort_scatter_block<R, true>(p, (int)blockIdx.x);
}

// ---------------------------------------------------------------- fields
template <typename R>
struct Field2Args {
  Fields2Dev<R> in, out;          // E^n, B^n -> E^{n+1}, B^{n+1}
  const long long* J[3];          // current of this step
  unsigned long long* Jnext[3];   // current of the next step, zeroed here
  long long* cont;                // [(nx + 1) ny] integer charge carried by the current
  double* flux;                   // [3][ny] per row: E_in, E_out_left, E_out_right
  long long* step_dev;            // device step counter, set to step + 1
  long long step;                 // this step (the laser clock)
  int nx, ny;
  R a, ha, dt;                    // dt/dx, dt/(2 dx), dt
  double dtd, dy;
  double sJ, sJz;                 // fixed point -> current density (Jx, Jy; Jz)
  double ay, az;                  // incident amplitude per component
  double tr, tf, tl;              // envelope (1/omega)
  double waist, yc;               // transverse profile exp(-((y - yc) / waist)^2); waist 0: flat
};

__device__ __forceinline__ double profile2(double y, double yc, double waist) {
  if (waist <= 0.0) return 1.0;
  const double u = (y - yc) / waist;
  return exp(-u * u);
}

// One Yee step on a tile of kFTX columns (X = node i and half-node h = X)
// by kFTY rows, with halos recomputed: the tile's E^n, B^n (two columns to
// the left and one to the right, one row below and two above) and J pass
// through LDS, then B^{n+1/2} (one column and row around the tile), E^{n+1}
// (one column to the left, one row above) and B^{n+1} at the tile.  Rows are
// periodic; every local row maps to global row (j0 - 1 + local) mod ny, so
// a period shorter than the tile just repeats.  The x-end positions apply the
// boundary guards at t_{n+1/2} and book the Poynting fluxes; each output
// cell updates its running charge and clears the next step's current.
#ifndef PIC2D_FIELD_TX
#define PIC2D_FIELD_TX 8
#endif
constexpr int kFTX = PIC2D_FIELD_TX, kFTY = 256 / PIC2D_FIELD_TX;
constexpr int kFAW = kFTX + 3, kFAH = kFTY + 3;  // E^n, B^n region
constexpr int kFW = kFTX + 2, kFH = kFTY + 2;    // J, B^{n+1/2}, E^{n+1} regions
static_assert(kFTX * kFTY == 256, "one thread per output cell");

template <typename R>
__global__ __launch_bounds__(256) void k_field2(Field2Args<R> p) {
  __shared__ R aEz[kFAW * kFAH], aEy[kFAW * kFAH], aBx[kFAW * kFAH];
  __shared__ R aEx[kFAW * kFAH], aBy[kFAW * kFAH], aBz[kFAW * kFAH];
  __shared__ long long sJ[3][kFW * kFH];
  __shared__ R hBz[kFW * kFH], hBy[kFW * kFH], hBx[kFW * kFH];
  __shared__ R nEx[kFW * kFH], nEy[kFW * kFH], nEz[kFW * kFH];
  __shared__ R gL[2][kFH], gR[2][kFH];          // guards (B_z, B_y) at h = 0 and h = nx + 1
  __shared__ double sIn[2][kFH];                // incident (E_y, E_z) per row
  const int t = threadIdx.x, n = p.nx, ny = p.ny;
  const int X0 = blockIdx.x * kFTX, j0 = blockIdx.y * kFTY;
  const R a = p.a, ha = p.ha, dt = p.dt;
  auto wrap = [&](int j) {
    j %= ny;
    return j < 0 ? j + ny : j;
  };
  // ---- load: E^n, B^n on columns X0-2 .. X0+kFTX, rows j0-1 .. j0+kFTY+1
  for (int e = t; e < kFAW * kFAH; e += 256) {
    const int lc = e / kFAH, lr = e - lc * kFAH;
    const int X = X0 - 2 + lc, gj = wrap(j0 - 1 + lr);
    const size_t gi = (size_t)X * ny + gj;
    const bool node = X >= 0 && X <= n, half = X >= 0 && X <= n + 1;
    const NH<R> v = node ? p.in.nh[gi] : NH<R>{R(0), R(0)};
    const HN<R> w = half ? p.in.hn[gi] : HN<R>{R(0), R(0)};
    aEz[e] = node ? p.in.ez[gi] : R(0);
    aEy[e] = v.ey;
    aBx[e] = v.bx;
    aEx[e] = w.ex;
    aBy[e] = w.by;
    aBz[e] = half ? p.in.bz[gi] : R(0);
  }
  // ---- J on columns X0-1 .. X0+kFTX, rows j0-1 .. j0+kFTY
  for (int e = t; e < kFW * kFH; e += 256) {
    const int lc = e / kFH, lr = e - lc * kFH;
    const int X = X0 - 1 + lc, gj = wrap(j0 - 1 + lr);
    const bool half = X >= 0 && X <= n + 1;
    sJ[0][e] = half ? p.J[0][(size_t)X * ny + gj] : 0;
    sJ[1][e] = X <= n + 1 ? p.J[1][(size_t)(X + 1) * ny + gj] : 0;
    sJ[2][e] = X <= n + 1 ? p.J[2][(size_t)(X + 1) * ny + gj] : 0;
  }
  __syncthreads();
  // ---- B^{n+1/2} on columns X0-1 .. X0+kFTX, rows j0-1 .. j0+kFTY
  for (int e = t; e < kFW * kFH; e += 256) {
    const int lc = e / kFH, lr = e - lc * kFH;
    const int X = X0 - 1 + lc;
    const int A = (lc + 1) * kFAH + lr, Am = A - kFAH;  // (X, row) and (X - 1, row) in the E^n region
    R bz = aBz[A], by = aBy[A], bx = aBx[A];
    if (X >= 1 && X <= n) {
      bz -= ha * ((aEy[A] - aEy[Am]) - (aEx[A + 1] - aEx[A]));
      by += ha * (aEz[A] - aEz[Am]);
    }
    if (X >= 0 && X <= n) bx -= ha * (aEz[A + 1] - aEz[A]);
    hBz[e] = bz;
    hBy[e] = by;
    hBx[e] = bx;
  }
  __syncthreads();
  // ---- E^{n+1} on columns X0-1 .. X0+kFTX-1, rows j0 .. j0+kFTY (with the guards)
  const double th = ((double)p.step + 0.5) * p.dtd;
  const double env = envelope(th, p.tr, p.tf, p.tl);
  for (int e = t; e < (kFTX + 1) * (kFTY + 1); e += 256) {
    const int lcx = e / (kFTY + 1), lrx = e - lcx * (kFTY + 1);
    const int lc = lcx, lr = lrx + 1;  // in the (kFW, kFH) regions
    const int X = X0 - 1 + lc;
    const int H = lc * kFH + lr;       // (X, row) in the B, J and E^{n+1} regions
    const int A = (lc + 1) * kFAH + lr;
    const R jx = (R)((double)sJ[0][H] * p.sJ), jy = (R)((double)sJ[1][H] * p.sJ);
    const R jz = (R)((double)sJ[2][H] * p.sJz);
    nEx[H] = (X >= 1 && X <= n) ? aEx[A] + (a * (hBz[H] - hBz[H - 1]) - dt * jx) : aEx[A];
    if (X < 0 || X > n) continue;
    R bz0 = hBz[H], bz1 = hBz[H + kFH], by0 = hBy[H], by1 = hBy[H + kFH];
    const R ey = aEy[A], ez = aEz[A], d = R(1) + a;
    if (X == 0) {
      const int gj = wrap(j0 - 1 + lr);
      const double ey_in = p.ay * env * sin(th) * profile2((gj + 0.5) * p.dy, p.yc, p.waist);
      const double ez_in = p.az * env * cos(th) * profile2((double)gj * p.dy, p.yc, p.waist);
      bz0 = (R(4) * (R)ey_in - R(2) * ey - (R(1) - a) * bz1 + dt * jy) / d;
      by0 = (R(2) * ez - (R(1) - a) * by1 - dt * jz - R(4) * (R)ez_in) / d;
      gL[0][lr] = bz0;
      gL[1][lr] = by0;
      sIn[0][lr] = ey_in;
      sIn[1][lr] = ez_in;
    }
    if (X == n) {
      bz1 = (R(2) * ey - (R(1) - a) * bz0 - dt * jy) / d;
      by1 = (R(-2) * ez - (R(1) - a) * by0 + dt * jz) / d;
      gR[0][lr] = bz1;
      gR[1][lr] = by1;
    }
    nEy[H] = ey - (a * (bz1 - bz0) + dt * jy);
    nEz[H] = ez + (a * ((by1 - by0) - (hBx[H] - hBx[H - 1])) - dt * jz);
  }
  __syncthreads();
  // ---- B^{n+1}, outputs, bookkeeping: one thread per cell of the tile
  const int X = X0 + t / kFTY, j = j0 + (t % kFTY);
  if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0) *p.step_dev = p.step + 1;
  if (X > n + 1 || j >= ny) return;
  const int lc = X - X0 + 1, lr = j - j0 + 1;
  const int H = lc * kFH + lr, A = (lc + 1) * kFAH + lr;
  const size_t gi = (size_t)X * ny + j;
  R bz, by;
  if (X >= 1 && X <= n) {
    bz = hBz[H] - ha * ((nEy[H] - nEy[H - kFH]) - (nEx[H + 1] - nEx[H]));
    by = hBy[H] + ha * (nEz[H] - nEz[H - kFH]);
  } else {  // guards keep their t_{n+1/2} value
    bz = X == 0 ? gL[0][lr] : gR[0][lr];
    by = X == 0 ? gL[1][lr] : gR[1][lr];
  }
  p.out.bz[gi] = bz;
  p.out.hn[gi] = HN<R>{nEx[H], by};
  p.Jnext[0][gi] = 0ull;
  p.Jnext[1][gi] = 0ull;
  p.Jnext[2][gi] = 0ull;
  if (X == n + 1) {
    p.Jnext[1][gi + ny] = 0ull;
    p.Jnext[2][gi + ny] = 0ull;
    return;
  }
  // node i = X
  const R bx = hBx[H] - ha * (nEz[H + 1] - nEz[H]);
  p.out.ez[gi] = nEz[H];
  p.out.nh[gi] = NH<R>{nEy[H], bx};
  const long long div = (sJ[0][H + kFH] - sJ[0][H]) + (sJ[1][H] - sJ[1][H - 1]);
  p.cont[gi] -= div;
  if (X == 0) {
    const double ey_in = sIn[0][lr], ez_in = sIn[1][lr];
    const double eyl = 0.5 * ((double)aEy[A] + (double)nEy[H]), ezl = 0.5 * ((double)aEz[A] + (double)nEz[H]);
    const double bzl = 0.5 * ((double)gL[0][lr] + (double)hBz[H + kFH]);
    const double byl = 0.5 * ((double)gL[1][lr] + (double)hBy[H + kFH]);
    const double L1 = eyl - bzl, L2 = ezl + byl;
    p.flux[j] += p.dtd * p.dy * (ey_in * ey_in + ez_in * ez_in);
    p.flux[ny + j] += p.dtd * p.dy * 0.25 * (L1 * L1 + L2 * L2);
  }
  if (X == n) {
    const double eyr = 0.5 * ((double)aEy[A] + (double)nEy[H]), ezr = 0.5 * ((double)aEz[A] + (double)nEz[H]);
    const double bzr = 0.5 * ((double)hBz[H] + (double)gR[0][lr]);
    const double byr = 0.5 * ((double)hBy[H] + (double)gR[1][lr]);
    const double R1 = eyr + bzr, R2 = ezr - byr;
    p.flux[2 * ny + j] += p.dtd * p.dy * 0.25 * (R1 * R1 + R2 * R2);
  }
}

// One Yee step, column-marching form, for periods of at most kFMRows<R>
// rows: a work-group owns all ny rows (one thread each) of a strip of
// columns [Xs, Xe) and walks along x.  At column c it forms B^{n+1/2} at c,
// E^{n+1} at c - 1 and B^{n+1} at c - 2 (with the outputs, running charge
// and next current of that column), while the loads of column c + 1 are in
// flight.  Every value is read once, plus the three columns a strip shares
// with its neighbours.  The row neighbours j + 1 and j - 1 (periodic) pass
// through LDS slots indexed by row, double-buffered by column parity, so
// one barrier per column orders them.  The arithmetic is that of k_field2,
// term by term.
template <typename R>
constexpr int kFMRows = sizeof(R) == 4 ? 1024 : 512;

template <typename R>
__host__ __device__ constexpr size_t field2m_lds(int ny) {
  return 2 * (size_t)ny * (6 * sizeof(R) + sizeof(long long));
}

template <typename R>
__global__ __launch_bounds__(kFMRows<R>) void k_field2m(Field2Args<R> p) {
  extern __shared__ __align__(16) unsigned char fsm[];
  const int n = p.nx, ny = p.ny, j = threadIdx.x;
  const bool live = j < ny;
  const int jp = j + 1 >= ny ? 0 : j + 1, jm = !live ? 0 : (j == 0 ? ny - 1 : j - 1);
  // strip of this block: columns [Xs, Xe), widths differing by at most one
  const int nb = gridDim.x, s = blockIdx.x, ncol = n + 2;
  const int Xs = (int)((long long)s * ncol / nb), Xe = (int)((long long)(s + 1) * ncol / nb);
  if (s == 0 && j == 0) *p.step_dev = p.step + 1;
  R* xr = (R*)fsm;                                              // [2][6][ny]
  long long* xj = (long long*)(fsm + 2 * 6 * (size_t)ny * sizeof(R));  // [2][ny]
  const R a = p.a, ha = p.ha, dt = p.dt, z = R(0);
  // column state, by age at the top of the iteration for column c:
  R ex0 = z, ey0 = z, ez0 = z, bx0 = z, by0c = z, bz0c = z;   // E^n, B^n (c)
  R ex1 = z, ey1 = z, ez1 = z;                                // E^n (c - 1)
  R ey2 = z, ez2 = z;                                         // E^n (c - 2)
  R hbz1 = z, hby1 = z, hbx1 = z, hbz2 = z, hby2 = z, hbx2 = z;  // B^{n+1/2} (c - 1), (c - 2)
  R nex2 = z, ney2 = z, nez2 = z, ney3 = z, nez3 = z;        // E^{n+1} (c - 2), (c - 3)
  long long jc0 = 0, jc1 = 0, jc2 = 0;                        // J (c)
  long long jp0 = 0, jp1 = 0, jp2 = 0;                        // J (c - 1)
  long long jq0 = 0, jq1 = 0;                                 // J_x, J_y (c - 2)
  long long cn2 = 0;                                          // running charge (c - 2)
  R gl0 = z, gl1 = z, gr0 = z, gr1 = z;                       // x-end guards at t_{n+1/2}
  double ey_in = 0.0, ez_in = 0.0;
  // next column's loads
  R fez = z, fbz = z;
  NH<R> fnh{z, z};
  HN<R> fhn{z, z};
  long long fj0 = 0, fj1 = 0, fj2 = 0, fcn = 0;
  auto load_col = [&](int col) {
    const bool nd = col >= 0 && col <= n, hf = col >= 0 && col <= n + 1;
    const size_t gi = (size_t)(col < 0 ? 0 : col) * ny + j;
    fez = live && nd ? p.in.ez[gi] : z;
    fnh = live && nd ? p.in.nh[gi] : NH<R>{z, z};
    fhn = live && hf ? p.in.hn[gi] : HN<R>{z, z};
    fbz = live && hf ? p.in.bz[gi] : z;
    fj0 = live && hf ? p.J[0][gi] : 0;
    const bool jy = live && col >= -1 && col <= n + 1;
    const size_t gk = (size_t)(col + 1 < 0 ? 0 : col + 1) * ny + j;
    fj1 = jy ? p.J[1][gk] : 0;
    fj2 = jy ? p.J[2][gk] : 0;
  };
  load_col(Xs - 2);
  ex0 = fhn.ex; ey0 = fnh.ey; ez0 = fez; bx0 = fnh.bx; by0c = fhn.by; bz0c = fbz;
  jc0 = fj0; jc1 = fj1; jc2 = fj2;
  const double th = ((double)p.step + 0.5) * p.dtd;
  for (int c = Xs - 2; c <= Xe + 1; ++c) {
    // loads for the next iterations: E^n, B^n, J of column c + 1 (needed up
    // to column Xe), the running charge of column c - 1 (output next)
    if (c + 1 <= Xe) load_col(c + 1);
    const int xo = c - 1;  // output column of the next iteration
    fcn = live && xo >= Xs && xo < Xe && xo <= n ? p.cont[(size_t)xo * ny + j] : 0;
    // publish the values rows j - 1 and j + 1 take from this row
    R* X = xr + (size_t)(c & 1) * 6 * ny;
    long long* XJ = xj + (size_t)(c & 1) * ny;
    if (live) {
      X[j] = ex0;
      X[ny + j] = ez0;
      X[2 * ny + j] = hbz1;
      X[3 * ny + j] = hbx1;
      X[4 * ny + j] = nex2;
      X[5 * ny + j] = nez2;
      XJ[j] = jq1;
    }
    __syncthreads();
    const R exn = X[jp], ezn = X[ny + jp];           // E^n (c) at j + 1
    const R hbzm = X[2 * ny + jm], hbxm = X[3 * ny + jm];  // B^{n+1/2} (c - 1) at j - 1
    const R nexn = X[4 * ny + jp], nezn = X[5 * ny + jp];  // E^{n+1} (c - 2) at j + 1
    const long long j1m = XJ[jm];                    // J_y (c - 2) at j - 1
    // B^{n+1/2} at column c
    R hbz0 = bz0c, hby0 = by0c, hbx0 = bx0;
    if (c >= 1 && c <= n) {
      hbz0 -= ha * ((ey0 - ey1) - (exn - ex0));
      hby0 += ha * (ez0 - ez1);
    }
    if (c >= 0 && c <= n) hbx0 -= ha * (ezn - ez0);
    // E^{n+1} at column c - 1
    R nex1 = z, ney1 = z, nez1 = z;
    const int Xn = c - 1;
    if (Xn >= Xs - 1 && Xn <= Xe - 1) {
      const R jx = (R)((double)jp0 * p.sJ), jy = (R)((double)jp1 * p.sJ);
      const R jz = (R)((double)jp2 * p.sJz);
      nex1 = (Xn >= 1 && Xn <= n) ? ex1 + (a * (hbz1 - hbzm) - dt * jx) : ex1;
      if (Xn >= 0 && Xn <= n) {
        R bz0 = hbz1, bz1 = hbz0, by0 = hby1, by1 = hby0;
        const R ey = ey1, ez = ez1, d = R(1) + a;
        if (Xn == 0) {
          const double env = envelope(th, p.tr, p.tf, p.tl);
          ey_in = p.ay * env * sin(th) * profile2((j + 0.5) * p.dy, p.yc, p.waist);
          ez_in = p.az * env * cos(th) * profile2((double)j * p.dy, p.yc, p.waist);
          bz0 = (R(4) * (R)ey_in - R(2) * ey - (R(1) - a) * bz1 + dt * jy) / d;
          by0 = (R(2) * ez - (R(1) - a) * by1 - dt * jz - R(4) * (R)ez_in) / d;
          gl0 = bz0;
          gl1 = by0;
        }
        if (Xn == n) {
          bz1 = (R(2) * ey - (R(1) - a) * bz0 - dt * jy) / d;
          by1 = (R(-2) * ez - (R(1) - a) * by0 + dt * jz) / d;
          gr0 = bz1;
          gr1 = by1;
        }
        ney1 = ey - (a * (bz1 - bz0) + dt * jy);
        nez1 = ez + (a * ((by1 - by0) - (hbx1 - hbxm)) - dt * jz);
      }
    }
    // B^{n+1} and the outputs at column c - 2
    const int Xo = c - 2;
    if (live && Xo >= Xs && Xo < Xe) {
      const size_t gi = (size_t)Xo * ny + j;
      R bz, by;
      if (Xo >= 1 && Xo <= n) {
        bz = hbz2 - ha * ((ney2 - ney3) - (nexn - nex2));
        by = hby2 + ha * (nez2 - nez3);
      } else {  // guards keep their t_{n+1/2} value
        bz = Xo == 0 ? gl0 : gr0;
        by = Xo == 0 ? gl1 : gr1;
      }
      p.out.bz[gi] = bz;
      p.out.hn[gi] = HN<R>{nex2, by};
      p.Jnext[0][gi] = 0ull;
      p.Jnext[1][gi] = 0ull;
      p.Jnext[2][gi] = 0ull;
      if (Xo == n + 1) {
        p.Jnext[1][gi + ny] = 0ull;
        p.Jnext[2][gi + ny] = 0ull;
      } else {
        const R bx = hbx2 - ha * (nezn - nez2);
        p.out.ez[gi] = nez2;
        p.out.nh[gi] = NH<R>{ney2, bx};
        const long long div = (jp0 - jq0) + (jq1 - j1m);
        p.cont[gi] = cn2 - div;
        if (Xo == 0) {
          const double eyl = 0.5 * ((double)ey2 + (double)ney2), ezl = 0.5 * ((double)ez2 + (double)nez2);
          const double bzl = 0.5 * ((double)gl0 + (double)hbz1);
          const double byl = 0.5 * ((double)gl1 + (double)hby1);
          const double L1 = eyl - bzl, L2 = ezl + byl;
          p.flux[j] += p.dtd * p.dy * (ey_in * ey_in + ez_in * ez_in);
          p.flux[ny + j] += p.dtd * p.dy * 0.25 * (L1 * L1 + L2 * L2);
        }
        if (Xo == n) {
          const double eyr = 0.5 * ((double)ey2 + (double)ney2), ezr = 0.5 * ((double)ez2 + (double)nez2);
          const double bzr = 0.5 * ((double)hbz2 + (double)gr0);
          const double byr = 0.5 * ((double)hby2 + (double)gr1);
          const double R1 = eyr + bzr, R2 = ezr - byr;
          p.flux[2 * ny + j] += p.dtd * p.dy * 0.25 * (R1 * R1 + R2 * R2);
        }
      }
    }
    // age the column state by one
    ey2 = ey1; ez2 = ez1;
    ex1 = ex0; ey1 = ey0; ez1 = ez0;
    ex0 = fhn.ex; ey0 = fnh.ey; ez0 = fez; bx0 = fnh.bx; by0c = fhn.by; bz0c = fbz;
    hbz2 = hbz1; hby2 = hby1; hbx2 = hbx1;
    hbz1 = hbz0; hby1 = hby0; hbx1 = hbx0;
    ney3 = ney2; nez3 = nez2;
    nex2 = nex1; ney2 = ney1; nez2 = nez1;
    jq0 = jp0; jq1 = jp1;
    jp0 = jc0; jp1 = jc1; jp2 = jc2;
    jc0 = fj0; jc1 = fj1; jc2 = fj2;
    cn2 = fcn;
  }
}

// ---------------------------------------------------------------- init
// Quiet start: particle i of the foil (cells column by column, rows fastest;
// k = i mod ppc, kx = k / ppc_y, ky = k mod ppc_y) at offsets
// ((kx + 1/2) + jitter (U_2i - 1/2)) / ppc_x, ((ky + 1/2) + jitter (U_2i+1 - 1/2)) / ppc_y
template <typename R>
__global__ void k_init2(SpeciesDev<R> e, SpeciesDev<R> ion, long long n, int c0, int ny, int ysh,
                        int ppcx, int ppcy, unsigned long long seed, double jitter, R w) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ppc = ppcx * ppcy;
  const long long q = i / ppc;
  const int k = (int)(i - q * ppc);
  const int kx = k / ppcy, ky = k - kx * ppcy;
  const int ix = c0 + (int)(q / ny), iy = (int)(q % ny);
  const R U1 = (R)(splitmix64(seed, 2ull * (unsigned long long)i) >> 40) * R(1.0 / 16777216.0);
  const R U2 = (R)(splitmix64(seed, 2ull * (unsigned long long)i + 1ull) >> 40) * R(1.0 / 16777216.0);
  R ox = ((R)kx + R(0.5) + (R)jitter * (U1 - R(0.5))) / (R)ppcx;
  R oy = ((R)ky + R(0.5) + (R)jitter * (U2 - R(0.5))) / (R)ppcy;
  if (!(ox < R(1))) ox = R(0);
  if (!(oy < R(1))) oy = R(0);
  SpeciesDev<R> sp[2] = {e, ion};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    sp[s].cell[i] = (ix << ysh) | iy;
    sp[s].off[i] = ox;
    sp[s].oy[i] = oy;
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
constexpr int k2DiagBlocks = 512;

template <typename R>
struct Diag2Args {
  SpeciesDev<R> sp[2];
  const long long* count;
  Fields2Dev<R> f;
  const long long* cont;
  long long* rho;       // [(nx + 1) ny] integer charge of the particles, zeroed by the caller
  double* part;         // [6][k2DiagBlocks]: K_e, K_i, U_Ex, U_Et, U_B, gauss max
  long long* ipart;     // [3][k2DiagBlocks]: alive e, alive i, continuity max
  int nx, ny, ysh;
  double mass[2];
  int Z[2];
  R sw;
  double dx, srho;      // integer charge -> density
};

// kinetic energy, alive counts and the integer charge 2 qw S_x S_y
template <typename R>
__global__ __launch_bounds__(256) void k_diag2_particles(Diag2Args<R> p) {
  __shared__ double sh[4];
  const int s = blockIdx.x < k2DiagBlocks ? 0 : 1;
  const int b = blockIdx.x - s * k2DiagBlocks;
  const long long n = p.count[s];
  const SpeciesDev<R> sp = p.sp[s];
  const int ymask = (1 << p.ysh) - 1, ny = p.ny;
  double ke = 0.0;
  long long alive = 0;
  for (long long i = (long long)b * 256 + threadIdx.x; i < n; i += (long long)k2DiagBlocks * 256) {
    const int c = sp.cell[i];
    if (c == kDead) continue;
    const double ux = sp.ux[i], uy = sp.uy[i], uz = sp.uz[i];
    ke += (double)sp.w[i] * p.mass[s] * (sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0);
    alive += 1;
    const int ix = c >> p.ysh, iy = c & ymask, iy1 = iy + 1 == ny ? 0 : iy + 1;
    const long long qx = (long long)(sp.off[i] * R(k2One)), qy = (long long)(sp.oy[i] * R(k2One));
    const long long qw = 2ll * p.Z[s] * (long long)rint(sp.w[i] * p.sw);
    unsigned long long* r = (unsigned long long*)p.rho;
    const size_t c0 = (size_t)ix * ny, c1 = c0 + ny;
    atomicAdd(r + c0 + iy, (unsigned long long)(qw * (k2One - qx) * (k2One - qy)));
    atomicAdd(r + c0 + iy1, (unsigned long long)(qw * (k2One - qx) * qy));
    atomicAdd(r + c1 + iy, (unsigned long long)(qw * qx * (k2One - qy)));
    atomicAdd(r + c1 + iy1, (unsigned long long)(qw * qx * qy));
  }
  const double t = block_sum(ke, sh);
  __shared__ long long sa[4];
  const long long na = wave_sum((long long)alive);
  if ((threadIdx.x & 63) == 0) sa[threadIdx.x >> 6] = na;
  __syncthreads();
  if (threadIdx.x == 0) {
    p.part[s * k2DiagBlocks + b] = t;
    p.ipart[s * k2DiagBlocks + b] = sa[0] + sa[1] + sa[2] + sa[3];
  }
}

// field energies, Gauss residual from the fields and the particles' charge,
// and the largest difference between that charge and the one the current
// carried, over interior nodes (exact integers: expect 0)
template <typename R>
__global__ __launch_bounds__(256) void k_diag2_fields(Diag2Args<R> p) {
  __shared__ double sh[4];
  __shared__ long long sm[4];
  const int ny = p.ny, n = p.nx;
  double ux = 0.0, ue = 0.0, ub = 0.0, gmax = 0.0;
  long long cmax = 0;
  const long long tot = (long long)(n + 2) * ny;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < tot;
       t += (long long)k2DiagBlocks * 256) {
    const int X = (int)(t / ny), j = (int)(t - (long long)X * ny);
    const size_t c = (size_t)X * ny;
    if (X <= n) {
      const double wn = (X == 0 || X == n) ? 0.5 : 1.0;
      const NH<R> e = p.f.nh[c + j];
      const double ey = e.ey, ez = p.f.ez[c + j], bxv = e.bx;
      ue += wn * (ey * ey + ez * ez);
      ub += wn * bxv * bxv;
      if (X >= 1 && X <= n - 1) {
        // interior nodes: a particle removed at an x end leaves part of its
        // last shape on the end node, which the current never takes away
        long long dc = p.cont[c + j] - p.rho[c + j];
        dc = dc < 0 ? -dc : dc;
        cmax = dc > cmax ? dc : cmax;
        const int jm = j == 0 ? ny - 1 : j - 1;
        const double divE = ((double)p.f.hn[c + ny + j].ex - (double)p.f.hn[c + j].ex) / p.dx +
                            ((double)e.ey - (double)p.f.nh[c + jm].ey) / p.dx;
        const double r = fabs(divE - (double)p.rho[c + j] * p.srho);
        gmax = r > gmax ? r : gmax;
      }
    }
    if (X >= 1 && X <= n) {
      const HN<R> h = p.f.hn[c + j];
      const double exv = h.ex, byv = h.by, bzv = p.f.bz[c + j];
      ux += exv * exv;
      ub += byv * byv + bzv * bzv;
    }
  }
  const double a2 = 0.5 * p.dx * p.dx;
  const double t0 = block_sum(ux, sh), t1 = block_sum(ue, sh), t2 = block_sum(ub, sh);
  double g = gmax;
  long long cm = cmax;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double v = __shfl_xor(g, o);
    g = v > g ? v : g;
    const long long w = __shfl_xor(cm, o);
    cm = w > cm ? w : cm;
  }
  __shared__ double sg[4];
  if ((threadIdx.x & 63) == 0) {
    sg[threadIdx.x >> 6] = g;
    sm[threadIdx.x >> 6] = cm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double gm = 0.0;
    long long m = 0;
    for (int w = 0; w < 4; ++w) {
      gm = sg[w] > gm ? sg[w] : gm;
      m = sm[w] > m ? sm[w] : m;
    }
    p.part[2 * k2DiagBlocks + blockIdx.x] = a2 * t0;
    p.part[3 * k2DiagBlocks + blockIdx.x] = a2 * t1;
    p.part[4 * k2DiagBlocks + blockIdx.x] = a2 * t2;
    p.part[5 * k2DiagBlocks + blockIdx.x] = gm;
    p.ipart[2 * k2DiagBlocks + blockIdx.x] = m;
  }
}

struct Diag2OutDev {
  double U_Ex, U_Et, U_B, K_e, K_i, E_rad, E_esc, n_stiff, gauss, E_in, E_ol, E_or;
  long long cont_max, alive0, alive1;
};

__global__ __launch_bounds__(256) void k_diag2_final(const double* part, const long long* ipart,
                                                     const double* acc, int tiles,
                                                     const double* flux, int ny, Diag2OutDev* out) {
  __shared__ double sh[256];
  Diag2OutDev o{};
  o.K_e = fixed_sum(part, k2DiagBlocks, 1, 0, sh);
  o.K_i = fixed_sum(part + k2DiagBlocks, k2DiagBlocks, 1, 0, sh);
  o.U_Ex = fixed_sum(part + 2 * k2DiagBlocks, k2DiagBlocks, 1, 0, sh);
  o.U_Et = fixed_sum(part + 3 * k2DiagBlocks, k2DiagBlocks, 1, 0, sh);
  o.U_B = fixed_sum(part + 4 * k2DiagBlocks, k2DiagBlocks, 1, 0, sh);
  o.E_rad = fixed_sum(acc, tiles, 4, 0, sh);
  o.E_esc = fixed_sum(acc, tiles, 4, 1, sh) + fixed_sum(acc, tiles, 4, 2, sh);
  o.n_stiff = fixed_sum(acc, tiles, 4, 3, sh);
  o.E_in = fixed_sum(flux, ny, 1, 0, sh);
  o.E_ol = fixed_sum(flux + ny, ny, 1, 0, sh);
  o.E_or = fixed_sum(flux + 2 * ny, ny, 1, 0, sh);
  if (threadIdx.x == 0) {
    for (int b = 0; b < k2DiagBlocks; ++b) {
      o.alive0 += ipart[b];
      o.alive1 += ipart[k2DiagBlocks + b];
      o.cont_max = ipart[2 * k2DiagBlocks + b] > o.cont_max ? ipart[2 * k2DiagBlocks + b] : o.cont_max;
      o.gauss = part[5 * k2DiagBlocks + b] > o.gauss ? part[5 * k2DiagBlocks + b] : o.gauss;
    }
    *out = o;
  }
}

}  // namespace pic
