// Explicit forward-Euler finite-difference solver (Sec. 2.4.1) with the
// second-order Laplacian stencils of Sec. 2.2.2, on the real-space fields.
//
// Stencils (periodic wrap; axes are powers of two, so wrapping is a mask;
// all but the axis-wise ones need equal spacing h on every axis):
//   ST = 0  axis-wise central differences (5 points in 2D, 7 in 3D),
//           sum over axes of (f[-1] - 2 f + f[+1]) / h_a^2;
//   ST = 9  2D isotropic: (4 sum(edge neighbours) + sum(corners) - 20 f) / (6 h^2);
//   ST = 15 3D isotropic: (8 sum(face neighbours) + sum(corners) - 56 f) / (12 h^2);
//   ST = 19 3D isotropic: (2 sum(face neighbours) + sum(edge neighbours)
//           - 24 f) / (6 h^2);
//   ST = 21 (3D) isotropic: (4 sum(edge neighbours) - sum(corners) - 40 f) / (12 h^2);
//   ST = 27 3D isotropic: (14 sum(faces) + 3 sum(edges) + sum(corners)
//           - 128 f) / (30 h^2);
//   ST = 4  fourth-order axis-wise (the fourth-order family; 9 points in
//           2D, 13 in 3D): sum over axes of
//           (-f[-2] + 16 f[-1] - 30 f + 16 f[+1] - f[+2]) / (12 h_a^2);
//   ST = 17 2D fourth-order isotropic: (128 A1 + 16 D1 - 8 A2 - D2 - 540 f) / (120 h^2);
//   ST = 21 (2D) fourth-order isotropic: (52 A1 + 16 D1 - A2 - 2 K - 252 f) / (60 h^2)
// (A1, A2: axis neighbours at distance 1 and 2; D1, D2: diagonal ones at
// (+-1, +-1) and (+-2, +-2); K: the 8 at (+-1, +-2) and (+-2, +-1)).  The
// weights of each family follow from its moment conditions on its points:
// zero sum, second moment 2 per axis, and an error term of |k| only
// (second order: h^2 |k|^4 / 12; fourth order: vanishing fourth moments
// and h^4 |k|^6 / 90).
// The leading error of the isotropic stencils depends on |k| only.
//
// One launch applies one operation at every cell: where the grid tiles,
// a marching kernel (fd2_march_kernel, fd3_march_kernel: the rows or
// planes of the Laplacian's input held in LDS), else fd_kernel (a thread
// per R cells along y, x fastest across threads).  A step is one to three
// launches, by model (the forms of the right-hand sides are those of the
// equations of motion of Sec. 3):
//   FD_AC     psi' = psi + dt M (kappa L psi + c1 psi - c2 psi^3)
//   FD_GS     u' = u + dt (Du L u - u v^2 + F (1 - u)),
//             v' = v + dt (Dv L v + u v^2 - (F + k) v)
//   FD_MU_CH  mu = c2 psi^3 - c1 psi - kappa L psi
//   FD_UPD    q' = q + dt s L w                      (conserved update)
//   FD_LAP    a = L psi
//   FD_MU_PFC mu = (r + q0^4) psi + 2 q0^2 a + L a + g2 psi^2 + g3 psi^3
//   FD_MC     psi' = psi + dt (L psi + c1 psi - c2 psi^3 + 2 c5 psi m),
//             b = -L m - c3 m + c4 m^3 - c5 psi^2     (then m' = m + dt L b)
//   FD_CH     psi' = psi + dt M L mu with mu recomputed at every stencil
//             point from psi (FD_MU_CH and FD_UPD in one launch: the
//             neighbours' psi come from the caches, and the step moves two
//             arrays instead of five; same arithmetic, same bits)
//
// Equations read at run time (Sec. 2.4.2 split, stepped with Sec. 2.4.1)
// take fd_eq_kernel instead: field j's right-hand side
//   sum_p c_p L^p psi_j + L^p_j E_j(psi)
// is written as nested levels, v_D = c_D psi_j (+ E_j) and
//   v_k = c_k psi_j (+ E_j if p_j = k) + L v_{k+1},
// so that v_0 is the right-hand side.  One launch evaluates one level from
// the next (DEPTH = 1), which is read from the array the launch before it
// wrote, or evaluated pointwise from the fields when it is the top level;
// a level with no Laplacian below it is DEPTH = 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ss {

enum { FD_AC = 0, FD_GS = 1, FD_MU_CH = 2, FD_UPD = 3, FD_LAP = 4, FD_MU_PFC = 5, FD_MC = 6, FD_CH = 7 };

struct FDArgs {
  const void* in[2];
  void* out[2];
  int64_t nx, ny, nz;        // nz = 1 in 2D
  int lx, lxy;               // log2(nx), log2(nx * ny)
  double ih2[3];             // 1 / h_a^2 (x, y, z) for the axis-wise stencil
  double i6h2;               // 1 / (6 h^2) for the 9- and 19-point stencils
  double i30h2;              // 1 / (30 h^2) for the 27-point stencil
  double i12h2;              // 1 / (12 h^2) for the 15- and 21-point 3D stencils
  double i60h2;              // 1 / (60 h^2) for the 21-point 2D stencil
  double i120h2;             // 1 / (120 h^2) for the 17-point 2D stencil
  double dt;
  double p[6];               // operation coefficients
  int op;
};

// The stencil applied to at(dx, dy, dz), the value at offset (dx, dy, dz).
template <typename T, int DIM, int ST, typename AT>
__device__ __forceinline__ T fd_stencil(AT&& at, const FDArgs& a) {
  const T c = at(0, 0, 0);
  if constexpr (ST == 0) {
    T s = (at(-1, 0, 0) + at(1, 0, 0) - (T)2 * c) * (T)a.ih2[0] +
          (at(0, -1, 0) + at(0, 1, 0) - (T)2 * c) * (T)a.ih2[1];
    if constexpr (DIM == 3) s += (at(0, 0, -1) + at(0, 0, 1) - (T)2 * c) * (T)a.ih2[2];
    return s;
  } else if constexpr (ST == 4) {
    T s = (-(at(-2, 0, 0) + at(2, 0, 0)) + (T)16 * (at(-1, 0, 0) + at(1, 0, 0)) - (T)30 * c) * (T)a.ih2[0] +
          (-(at(0, -2, 0) + at(0, 2, 0)) + (T)16 * (at(0, -1, 0) + at(0, 1, 0)) - (T)30 * c) * (T)a.ih2[1];
    if constexpr (DIM == 3)
      s += (-(at(0, 0, -2) + at(0, 0, 2)) + (T)16 * (at(0, 0, -1) + at(0, 0, 1)) - (T)30 * c) * (T)a.ih2[2];
    return s * ((T)1 / (T)12);
  } else if constexpr (DIM == 2 && ST == 9) {
    const T edge = at(-1, 0, 0) + at(1, 0, 0) + at(0, -1, 0) + at(0, 1, 0);
    const T corner = at(-1, -1, 0) + at(1, -1, 0) + at(-1, 1, 0) + at(1, 1, 0);
    return ((T)4 * edge + corner - (T)20 * c) * (T)a.i6h2;
  } else if constexpr (DIM == 2) {   // 17 or 21: fourth-order isotropic
    const T a1 = at(-1, 0, 0) + at(1, 0, 0) + at(0, -1, 0) + at(0, 1, 0);
    const T d1 = at(-1, -1, 0) + at(1, -1, 0) + at(-1, 1, 0) + at(1, 1, 0);
    const T a2 = at(-2, 0, 0) + at(2, 0, 0) + at(0, -2, 0) + at(0, 2, 0);
    if constexpr (ST == 17) {
      const T d2 = at(-2, -2, 0) + at(2, -2, 0) + at(-2, 2, 0) + at(2, 2, 0);
      return ((T)128 * a1 + (T)16 * d1 - (T)8 * a2 - d2 - (T)540 * c) * (T)a.i120h2;
    } else {
      const T kn = at(-1, -2, 0) + at(1, -2, 0) + at(-2, -1, 0) + at(2, -1, 0) +
                   at(-2, 1, 0) + at(2, 1, 0) + at(-1, 2, 0) + at(1, 2, 0);
      return ((T)52 * a1 + (T)16 * d1 - a2 - (T)2 * kn - (T)252 * c) * (T)a.i60h2;
    }
  } else {
    auto faces = [&]() {
      return at(-1, 0, 0) + at(1, 0, 0) + at(0, -1, 0) + at(0, 1, 0) + at(0, 0, -1) + at(0, 0, 1);
    };
    auto edges = [&]() {
      return at(-1, -1, 0) + at(1, -1, 0) + at(-1, 1, 0) + at(1, 1, 0) +
             at(-1, 0, -1) + at(1, 0, -1) + at(-1, 0, 1) + at(1, 0, 1) +
             at(0, -1, -1) + at(0, 1, -1) + at(0, -1, 1) + at(0, 1, 1);
    };
    auto corners = [&]() {
      return at(-1, -1, -1) + at(1, -1, -1) + at(-1, 1, -1) + at(1, 1, -1) +
             at(-1, -1, 1) + at(1, -1, 1) + at(-1, 1, 1) + at(1, 1, 1);
    };
    if constexpr (ST == 15) {
      return ((T)8 * faces() + corners() - (T)56 * c) * (T)a.i12h2;
    } else if constexpr (ST == 19) {
      return ((T)2 * faces() + edges() - (T)24 * c) * (T)a.i6h2;
    } else if constexpr (ST == 21) {
      return ((T)4 * edges() - corners() - (T)40 * c) * (T)a.i12h2;
    } else {   // 27
      return ((T)14 * faces() + (T)3 * edges() + corners() - (T)128 * c) * (T)a.i30h2;
    }
  }
}

// Cells of rim the stencil needs around a cell: two for the fourth-order
// family (and its knight and (2, 2) points), one otherwise.
constexpr int fd_halo(int dim, int st) { return (st == 4 || (dim == 2 && (st == 17 || st == 21))) ? 2 : 1; }

// The stencil applied to array f around cell (x, y, z) (periodic wrap;
// x, y, z may lie one or two cells outside the grid).
template <typename T, int DIM, int ST>
__device__ __forceinline__ T fd_lap(const T* __restrict__ f, int64_t x, int64_t y, int64_t z, const FDArgs& a) {
  const int64_t mx = a.nx - 1, my = a.ny - 1, mz = a.nz - 1;
  auto at = [&](int64_t dx, int64_t dy, int64_t dz) -> T {
    return f[((((z + dz) & mz) * a.ny + ((y + dy) & my)) << a.lx) + ((x + dx) & mx)];
  };
  return fd_stencil<T, DIM, ST>(at, a);
}

// Cahn-Hilliard chemical potential at one cell (the FD_MU_CH expression).
template <typename T, int DIM, int ST>
__device__ __forceinline__ T fd_mu_ch(const T* __restrict__ f, int64_t x, int64_t y, int64_t z, const FDArgs& a) {
  const T kap = (T)a.p[1], c1 = (T)a.p[2], c2 = (T)a.p[3];
  const int64_t i = ((((z & (a.nz - 1)) * a.ny + (y & (a.ny - 1))) << a.lx) + (x & (a.nx - 1)));
  const T q = f[i];
  return c2 * q * q * q - c1 * q - kap * fd_lap<T, DIM, ST>(f, x, y, z, a);
}

// The explicit terms of field j, E = sum_k f1^k sum_i a[j][k][i] f0^i,
// i <= du[j][k], k <= dv[j] (Horner in f0 inside Horner in f1), read from
// the kernel arguments by every lane at the same addresses (scalar loads:
// the loop bounds and guards are uniform branches).
struct FDEqTab {
  int dv[2];
  int du[2][8];
  double a[2][8][8];
  float af[2][8][8];
};

struct FDEq {
  int nj;               // fields this launch computes (1 or 2)
  int j[2];             // which fields
  int fin;              // 1: out = psi_j + dt v_0; 0: out = v_0
  double cl[2][2];      // coefficient of psi_j at nested level d (0: the output)
  int el[2][2];         // 1: E_j is added at nested level d
  const void* w[2];     // deepest level from this array, or null: pointwise
  void* out[2];
  FDEqTab tab;
};

template <typename T>
struct FDEqSlot {
  const T* f0;          // the fields
  const T* f1;
  const T* fj;          // field j
  const T* w;
  T cl[2];
  int el[2];
  int j;
};

template <typename T>
__device__ __forceinline__ T fd_eq_E(const FDEqTab* tb, int j, T u, T v) {
  T acc = (T)0;
  const int dv = tb->dv[j];
#pragma unroll 1
  for (int k = dv; k >= 0; --k) {
    const int dk = tb->du[j][k];
    T c[8];   // the row, read whole ahead of the guards
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = sizeof(T) == 8 ? (T)tb->a[j][k][i] : (T)tb->af[j][k][i];
    T h = (T)0;
#pragma unroll
    for (int i = 7; i >= 0; --i)
      if (i <= dk) h = h * u + c[i];
    acc = acc * v + h;
  }
  return acc;
}

// The axis-wise Laplacian of E_j around (x, y, z): E at the 2 DIM + 1
// points evaluated together (one pass over the table serves every point).
template <typename T, int DIM, int NF>
__device__ __forceinline__ T fd_eq_lapE(const FDArgs& a, const FDEqTab* tb, const FDEqSlot<T>& sl,
                                        int64_t x, int64_t y, int64_t z) {
  constexpr int P = 2 * DIM + 1;
  const int64_t mx = a.nx - 1, my = a.ny - 1, mz = a.nz - 1;
  T u[P], w[P], acc[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int ax = (p - 1) >> 1;                      // axis of point p (p > 0)
    const int64_t o = p == 0 ? 0 : ((p & 1) ? -1 : 1);
    const int64_t xx = x + (ax == 0 ? o : 0), yy = y + (ax == 1 ? o : 0), zz = z + (ax == 2 ? o : 0);
    const int64_t i = ((((zz & mz) * a.ny + (yy & my)) << a.lx) + (xx & mx));
    u[p] = sl.f0[i];
    w[p] = NF == 2 ? sl.f1[i] : (T)0;
    acc[p] = (T)0;
  }
  const int j = sl.j;
  const int dv = tb->dv[j];
#pragma unroll 1
  for (int k = dv; k >= 0; --k) {
    const int dk = tb->du[j][k];
    T c[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = sizeof(T) == 8 ? (T)tb->a[j][k][i] : (T)tb->af[j][k][i];
    T h[P];
#pragma unroll
    for (int p = 0; p < P; ++p) h[p] = (T)0;
#pragma unroll
    for (int i = 7; i >= 0; --i)
      if (i <= dk) {
#pragma unroll
        for (int p = 0; p < P; ++p) h[p] = h[p] * u[p] + c[i];
      }
#pragma unroll
    for (int p = 0; p < P; ++p) acc[p] = acc[p] * w[p] + h[p];
  }
  T s = (acc[1] + acc[2] - (T)2 * acc[0]) * (T)a.ih2[0] + (acc[3] + acc[4] - (T)2 * acc[0]) * (T)a.ih2[1];
  if constexpr (DIM == 3) s += (acc[5] + acc[6] - (T)2 * acc[0]) * (T)a.ih2[2];
  return s;
}

// Nested level D at cell (x, y, z) (coordinates may lie outside the grid:
// they wrap).  LW: the deepest level comes from the array w; NF fields.
// The loads do not depend on the coefficients, so that a stencil's loads
// issue together.  E_j enters at the centre (D = 0) directly and, with
// the axis-wise stencil, one level down as the Laplacian of E evaluated at
// the stencil's points together (the launches of the wider stencils put E
// at a level of their own, always the centre).
template <typename T, int DIM, int ST, int D, int DEPTH, bool LW, int NF>
__device__ __forceinline__ T fd_eq_level(const FDArgs& a, const FDEqTab* tb, const FDEqSlot<T>& sl,
                                         int64_t x, int64_t y, int64_t z) {
  const int64_t i = ((((z & (a.nz - 1)) * a.ny + (y & (a.ny - 1))) << a.lx) + (x & (a.nx - 1)));
  if constexpr (D == DEPTH && LW) {
    return sl.w[i];
  } else {
    const T u = sl.f0[i], w = NF == 2 ? sl.f1[i] : (T)0;
    T v = sl.cl[D] * (NF == 1 || sl.j == 0 ? u : w);
    if constexpr (D == 0)
      if (sl.el[0]) v += fd_eq_E<T>(tb, sl.j, u, w);
    if constexpr (D < DEPTH) {
      auto next = [&](int64_t dx, int64_t dy, int64_t dz) -> T {
        return fd_eq_level<T, DIM, ST, D + 1, DEPTH, LW, NF>(a, tb, sl, x + dx, y + dy, z + dz);
      };
      v += fd_stencil<T, DIM, ST>(next, a);
      if constexpr (ST == 0 && !(LW && D + 1 == DEPTH))
        if (sl.el[D + 1]) v += fd_eq_lapE<T, DIM, NF>(a, tb, sl, x, y, z);
    }
    return v;
  }
}

template <typename T, int DIM, int ST, int DEPTH, bool LW, int NF, int R>
__global__ void __launch_bounds__(256) fd_eq_kernel(FDArgs a, FDEq q) {
  const FDEqTab* tb = &q.tab;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t * R >= (a.nx * a.ny * a.nz)) return;
  constexpr int LR = R == 1 ? 0 : R == 2 ? 1 : R == 4 ? 2 : 3;
  const int64_t x = t & (a.nx - 1);
  const int64_t row = t >> a.lx;                          // over (ny / R) * nz
  const int64_t y0 = (row & ((a.ny >> LR) - 1)) << LR;
  const int64_t z = row >> (a.lxy - a.lx - LR);
  for (int s = 0; s < q.nj; ++s) {
    FDEqSlot<T> sl;
    sl.f0 = (const T*)a.in[0];
    sl.f1 = (const T*)a.in[1];
    sl.w = (const T*)q.w[s];
    sl.j = q.j[s];
    sl.fj = sl.j == 0 ? sl.f0 : sl.f1;
    for (int d = 0; d < 2; ++d) {
      sl.cl[d] = (T)q.cl[s][d];
      sl.el[d] = q.el[s][d];
    }
    // the thread's R cells along y, unrolled in one block (shared loads once)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t y = y0 + r;
      const int64_t i = (((z * a.ny) + y) << a.lx) + x;
      T v = fd_eq_level<T, DIM, ST, 0, DEPTH, LW, NF>(a, tb, sl, x, y, z);
      if (q.fin) v = sl.fj[i] + (T)a.dt * v;
      ((T*)q.out[s])[i] = v;
    }
  }
}

// A thread steps R consecutive cells along y (same x, same z): the loads
// that neighbouring cells share are issued once (R divides ny; ny >= 8).
// OP is a template parameter: each kernel holds the registers of its own
// operation only.
template <typename T, int DIM, int ST, int R, int OP>
__global__ void __launch_bounds__(256) fd_kernel(FDArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t * R >= (a.nx * a.ny * a.nz)) return;
  constexpr int LR = R == 1 ? 0 : R == 2 ? 1 : R == 4 ? 2 : 3;
  const int64_t x = t & (a.nx - 1);
  const int64_t row = t >> a.lx;                          // over (ny / R) * nz
  const int64_t y0 = (row & ((a.ny >> LR) - 1)) << LR;
  const int64_t z = row >> (a.lxy - a.lx - LR);
  const T* in0 = (const T*)a.in[0];
  const T* in1 = (const T*)a.in[1];
  T* out0 = (T*)a.out[0];
  T* out1 = (T*)a.out[1];
  const T dt = (T)a.dt;
  // the operation's body over the thread's R cells, unrolled in one block
  auto cells = [&](auto&& body) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t y = y0 + r;
      body((((z * a.ny) + y) << a.lx) + x, y);
    }
  };
  if constexpr (OP == FD_AC) {
    const T M = (T)a.p[0], kap = (T)a.p[1], c1 = (T)a.p[2], c2 = (T)a.p[3];
    cells([&](int64_t i, int64_t y) {
      const T q = in0[i];
      out0[i] = q + dt * (M * (kap * fd_lap<T, DIM, ST>(in0, x, y, z, a) + c1 * q - c2 * q * q * q));
    });
  } else if constexpr (OP == FD_GS) {
    const T du = (T)a.p[0], dv = (T)a.p[1], F = (T)a.p[2], kk = (T)a.p[3];
    cells([&](int64_t i, int64_t y) {
      const T u = in0[i], v = in1[i];
      const T uvv = u * v * v;
      out0[i] = u + dt * (du * fd_lap<T, DIM, ST>(in0, x, y, z, a) - uvv + F * ((T)1 - u));
      out1[i] = v + dt * (dv * fd_lap<T, DIM, ST>(in1, x, y, z, a) + uvv - (F + kk) * v);
    });
  } else if constexpr (OP == FD_MU_CH) {
    const T kap = (T)a.p[1], c1 = (T)a.p[2], c2 = (T)a.p[3];
    cells([&](int64_t i, int64_t y) {
      const T q = in0[i];
      out0[i] = c2 * q * q * q - c1 * q - kap * fd_lap<T, DIM, ST>(in0, x, y, z, a);
    });
  } else if constexpr (OP == FD_UPD) {
    const T s0 = (T)a.p[0];
    cells([&](int64_t i, int64_t y) { out0[i] = in0[i] + dt * (s0 * fd_lap<T, DIM, ST>(in1, x, y, z, a)); });
  } else if constexpr (OP == FD_LAP) {
    cells([&](int64_t i, int64_t y) { out0[i] = fd_lap<T, DIM, ST>(in0, x, y, z, a); });
  } else if constexpr (OP == FD_MU_PFC) {
    const T r = (T)a.p[0], q0 = (T)a.p[1], g2 = (T)a.p[2], g3 = (T)a.p[3];
    const T q02 = q0 * q0;
    cells([&](int64_t i, int64_t y) {
      const T q = in0[i], lq = in1[i];
      out0[i] = (r + q02 * q02) * q + (T)2 * q02 * lq + fd_lap<T, DIM, ST>(in1, x, y, z, a) + g2 * q * q +
                g3 * q * q * q;
    });
  } else if constexpr (OP == FD_CH) {
    const T M = (T)a.p[0];
    cells([&](int64_t i, int64_t y) {
      auto mu_at = [&](int64_t dx, int64_t dy, int64_t dz) -> T {
        return fd_mu_ch<T, DIM, ST>(in0, x + dx, y + dy, z + dz, a);
      };
      out0[i] = in0[i] + dt * (M * fd_stencil<T, DIM, ST>(mu_at, a));
    });
  } else {  // FD_MC
    const T c1 = (T)a.p[0], c2 = (T)a.p[1], c3 = (T)a.p[2], c4 = (T)a.p[3], c5 = (T)a.p[4];
    cells([&](int64_t i, int64_t y) {
      const T q = in0[i], m = in1[i];
      out0[i] = q + dt * (fd_lap<T, DIM, ST>(in0, x, y, z, a) + c1 * q - c2 * q * q * q + (T)2 * c5 * q * m);
      out1[i] = -fd_lap<T, DIM, ST>(in1, x, y, z, a) - c3 * m + c4 * m * m * m - c5 * q * q;
    });
  }
}

// 3D stencils: a 64 x 4 block of threads marches along z over ZC planes,
// keeping the 2 HALO + 1 planes z - HALO .. z + HALO of the Laplacian's
// input (of both fields for Gray-Scott and Model C; with a HALO-cell rim)
// in LDS, so that a cell's neighbours are read from LDS and the input is read
// from memory about once (HALO = 1: 7, 15, 19, 21 and 27 points; 2: fourth order).
// Needs nx % 64, ny % 4 and nz % ZC to be 0 (the host falls back to
// fd_kernel otherwise).
constexpr int FD3_BX = 64, FD3_BY = 4, FD3_ZC = 8;   // 8 planes a block: measured faster than 16 or 32 (more blocks in flight)
// rows per thread: two (tiles of 64 x 8, a thinner rim) for the axis-wise
// and fourth-order stencils, one for the 19- and 27-point ones (measured:
// CH 256^3 axis-wise 162 -> 148 us per step, 19-point 165 -> 170)
constexpr int fd3_rows(int st) { return (st == 0 || st == 4) ? 2 : 1; }

template <typename T, int ST, int OP, int HALO>
__global__ void __launch_bounds__(256) fd3_march_kernel(FDArgs a) {
  constexpr int RY = fd3_rows(ST), TY = FD3_BY * RY;   // a thread's rows ty + FD3_BY r, r < RY
  constexpr int W = FD3_BX + 2 * HALO, H = TY + 2 * HALO, NP = 2 * HALO + 1;
  constexpr bool LAP1 = OP == FD_UPD || OP == FD_MU_PFC;   // the Laplacian of in1
  constexpr int NS = (OP == FD_GS || OP == FD_MC) ? 2 : 1;  // arrays in LDS (Laplacians taken)
  __shared__ T pl[NS][NP][H][W];
  const int tid = threadIdx.x, tx = tid & (FD3_BX - 1), ty = tid / FD3_BX;
  const int64_t nbx = a.nx / FD3_BX, nby = a.ny / TY;
  int64_t b = blockIdx.x;
  const int64_t bx = b % nbx;
  b /= nbx;
  const int64_t by = b % nby, bz = b / nby;
  const int64_t x0 = bx * FD3_BX, y0 = by * TY, z0 = bz * FD3_ZC;
  const int64_t mx = a.nx - 1, my = a.ny - 1, mz = a.nz - 1;
  const T* in0 = (const T*)a.in[0];
  const T* in1 = (const T*)a.in[1];
  const T* const srcs[2] = {LAP1 ? in1 : in0, in1};
  T* out0 = (T*)a.out[0];
  T* out1 = (T*)a.out[1];
  // a plane's H x W values, NV per thread: read into registers (the next
  // plane's read is in flight while the current plane is computed), then
  // stored to its LDS slot
  constexpr int NV = (H * W + 255) / 256;
  T nxt[NS][NV];
  auto fetch_plane = [&](int64_t z) {
    const int64_t zo = (z & mz) * a.ny;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int p = tid + 256 * v;
      if (p < H * W) {
        const int ly = p / W, lx = p - ly * W;
        const int64_t gx = (x0 + lx - HALO) & mx, gy = (y0 + ly - HALO) & my;
#pragma unroll
        for (int n = 0; n < NS; ++n) nxt[n][v] = srcs[n][((zo + gy) << a.lx) + gx];
      }
    }
  };
  auto store_plane = [&](int slot) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int p = tid + 256 * v;
      if (p < H * W) {
        const int ly = p / W, lx = p - ly * W;
#pragma unroll
        for (int n = 0; n < NS; ++n) pl[n][slot][ly][lx] = nxt[n][v];
      }
    }
  };
  // plane z + dz of iteration k sits in slot (k + HALO + dz) % NP
  for (int j = 0; j < 2 * HALO; ++j) {
    fetch_plane(z0 - HALO + j);
    store_plane(j);
  }
  fetch_plane(z0 + HALO);
  const T dt = (T)a.dt;
  for (int k = 0; k < FD3_ZC; ++k) {
    const int64_t z = z0 + k;
    int64_t i[RY];
    T qg[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      i[r] = (((z * a.ny) + y0 + ty + FD3_BY * r) << a.lx) + x0 + tx;
      // a centre value of the other array, read ahead of the barrier (the
      // Laplacian's input is in LDS)
      qg[r] = (OP == FD_UPD || OP == FD_MU_PFC) ? in0[i[r]] : (T)0;
    }
    store_plane((k + 2 * HALO) % NP);
    if (k + 1 < FD3_ZC) fetch_plane(z + HALO + 1);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int yl = ty + FD3_BY * r + HALO;
      auto at = [&](int64_t dx, int64_t dy, int64_t dz) -> T {
        return pl[0][(k + HALO + (int)dz) % NP][yl + dy][tx + HALO + dx];
      };
      auto at1 = [&](int64_t dx, int64_t dy, int64_t dz) -> T {
        return pl[NS - 1][(k + HALO + (int)dz) % NP][yl + dy][tx + HALO + dx];
      };
      const T lap = fd_stencil<T, 3, ST>(at, a);
      const T c = at(0, 0, 0);
      const T q = (OP == FD_UPD || OP == FD_MU_PFC) ? qg[r] : c;   // psi
      const T lq = c;                                             // FD_MU_PFC: L psi
      const int64_t ii = i[r];
      if constexpr (OP == FD_AC) {
        const T M = (T)a.p[0], kap = (T)a.p[1], c1 = (T)a.p[2], c2 = (T)a.p[3];
        out0[ii] = q + dt * (M * (kap * lap + c1 * q - c2 * q * q * q));
      } else if constexpr (OP == FD_MU_CH) {
        const T kap = (T)a.p[1], c1 = (T)a.p[2], c2 = (T)a.p[3];
        out0[ii] = c2 * q * q * q - c1 * q - kap * lap;
      } else if constexpr (OP == FD_UPD) {
        out0[ii] = q + dt * ((T)a.p[0] * lap);
      } else if constexpr (OP == FD_LAP) {
        out0[ii] = lap;
      } else if constexpr (OP == FD_MU_PFC) {
        const T r0 = (T)a.p[0], q0 = (T)a.p[1], g2 = (T)a.p[2], g3 = (T)a.p[3];
        const T q02 = q0 * q0;
        out0[ii] = (r0 + q02 * q02) * q + (T)2 * q02 * lq + lap + g2 * q * q + g3 * q * q * q;
      } else if constexpr (OP == FD_GS) {
        const T du = (T)a.p[0], dv = (T)a.p[1], F = (T)a.p[2], kk = (T)a.p[3];
        const T u = c, v = at1(0, 0, 0), lap1 = fd_stencil<T, 3, ST>(at1, a);
        const T uvv = u * v * v;
        out0[ii] = u + dt * (du * lap - uvv + F * ((T)1 - u));
        out1[ii] = v + dt * (dv * lap1 + uvv - (F + kk) * v);
      } else {   // FD_MC
        const T c1 = (T)a.p[0], c2 = (T)a.p[1], c3 = (T)a.p[2], c4 = (T)a.p[3], c5 = (T)a.p[4];
        const T m = at1(0, 0, 0), lap1 = fd_stencil<T, 3, ST>(at1, a);
        out0[ii] = c + dt * (lap + c1 * c - c2 * c * c * c + (T)2 * c5 * c * m);
        out1[ii] = -lap1 - c3 * m + c4 * m * m * m - c5 * c * c;
      }
    }
    __syncthreads();   // the next iteration overwrites the plane z - HALO
  }
}

// The 2D form: a block of 256 threads along x marches along y over YC
// rows, keeping the rows y - HALO .. y + HALO of the Laplacian's input
// (of both fields for Gray-Scott and Model C; with a HALO-cell rim) in LDS; the next row is read into registers
// while the current one is computed.  Needs nx % 256 == 0 and ny % YC == 0.
constexpr int FD2_BX = 256, FD2_YC = 8;

template <typename T, int ST, int OP, int HALO>
__global__ void __launch_bounds__(256) fd2_march_kernel(FDArgs a) {
  constexpr int W = FD2_BX + 2 * HALO, NP = 2 * HALO + 1;
  constexpr bool LAP1 = OP == FD_UPD || OP == FD_MU_PFC;   // the Laplacian of in1
  constexpr int NS = (OP == FD_GS || OP == FD_MC) ? 2 : 1;  // arrays in LDS (Laplacians taken)
  __shared__ T pl[NS][NP][W];
  const int tid = threadIdx.x;
  const int64_t nbx = a.nx / FD2_BX;
  const int64_t bx = blockIdx.x % nbx, by = blockIdx.x / nbx;
  const int64_t x0 = bx * FD2_BX, y0 = by * FD2_YC;
  const int64_t mx = a.nx - 1, my = a.ny - 1;
  const T* in0 = (const T*)a.in[0];
  const T* in1 = (const T*)a.in[1];
  const T* const srcs[2] = {LAP1 ? in1 : in0, in1};
  T* out0 = (T*)a.out[0];
  T* out1 = (T*)a.out[1];
  constexpr int NV = (W + 255) / 256;
  T nxt[NS][NV];
  auto fetch_row = [&](int64_t y) {
    const int64_t yo = (y & my) << a.lx;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int p = tid + 256 * v;
      if (p < W) {
#pragma unroll
        for (int n = 0; n < NS; ++n) nxt[n][v] = srcs[n][yo + ((x0 + p - HALO) & mx)];
      }
    }
  };
  auto store_row = [&](int slot) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int p = tid + 256 * v;
      if (p < W) {
#pragma unroll
        for (int n = 0; n < NS; ++n) pl[n][slot][p] = nxt[n][v];
      }
    }
  };
  // row y + dy of iteration k sits in slot (k + HALO + dy) % NP
  for (int j = 0; j < 2 * HALO; ++j) {
    fetch_row(y0 - HALO + j);
    store_row(j);
  }
  fetch_row(y0 + HALO);
  const T dt = (T)a.dt;
  for (int k = 0; k < FD2_YC; ++k) {
    const int64_t y = y0 + k;
    const int64_t i = (y << a.lx) + x0 + tid;
    const T qg = (OP == FD_UPD || OP == FD_MU_PFC) ? in0[i] : (T)0;
    store_row((k + 2 * HALO) % NP);
    if (k + 1 < FD2_YC) fetch_row(y + HALO + 1);
    __syncthreads();
    auto at = [&](int64_t dx, int64_t dy, int64_t) -> T {
      return pl[0][(k + HALO + (int)dy) % NP][tid + HALO + dx];
    };
    auto at1 = [&](int64_t dx, int64_t dy, int64_t) -> T {
      return pl[NS - 1][(k + HALO + (int)dy) % NP][tid + HALO + dx];
    };
    const T lap = fd_stencil<T, 2, ST>(at, a);
    const T c = at(0, 0, 0);
    const T q = (OP == FD_UPD || OP == FD_MU_PFC) ? qg : c;   // psi
    const T lq = c;                                          // FD_MU_PFC: L psi
    if constexpr (OP == FD_AC) {
      const T M = (T)a.p[0], kap = (T)a.p[1], c1 = (T)a.p[2], c2 = (T)a.p[3];
      out0[i] = q + dt * (M * (kap * lap + c1 * q - c2 * q * q * q));
    } else if constexpr (OP == FD_MU_CH) {
      const T kap = (T)a.p[1], c1 = (T)a.p[2], c2 = (T)a.p[3];
      out0[i] = c2 * q * q * q - c1 * q - kap * lap;
    } else if constexpr (OP == FD_UPD) {
      out0[i] = q + dt * ((T)a.p[0] * lap);
    } else if constexpr (OP == FD_LAP) {
      out0[i] = lap;
    } else if constexpr (OP == FD_MU_PFC) {
      const T r = (T)a.p[0], q0 = (T)a.p[1], g2 = (T)a.p[2], g3 = (T)a.p[3];
      const T q02 = q0 * q0;
      out0[i] = (r + q02 * q02) * q + (T)2 * q02 * lq + lap + g2 * q * q + g3 * q * q * q;
    } else if constexpr (OP == FD_GS) {
      const T du = (T)a.p[0], dv = (T)a.p[1], F = (T)a.p[2], kk = (T)a.p[3];
      const T u = c, v = at1(0, 0, 0), lap1 = fd_stencil<T, 2, ST>(at1, a);
      const T uvv = u * v * v;
      out0[i] = u + dt * (du * lap - uvv + F * ((T)1 - u));
      out1[i] = v + dt * (dv * lap1 + uvv - (F + kk) * v);
    } else {   // FD_MC
      const T c1 = (T)a.p[0], c2 = (T)a.p[1], c3 = (T)a.p[2], c4 = (T)a.p[3], c5 = (T)a.p[4];
      const T m = at1(0, 0, 0), lap1 = fd_stencil<T, 2, ST>(at1, a);
      out0[i] = c + dt * (lap + c1 * c - c2 * c * c * c + (T)2 * c5 * c * m);
      out1[i] = -lap1 - c3 * m + c4 * m * m * m - c5 * c * c;
    }
    __syncthreads();   // the next iteration overwrites the row y - HALO
  }
}

// One level of an equation read at run time, v_0 = c_0 psi_j (+ E_j) +
// L v_1, with the marching scheme of the kernels above (2D: 256 threads
// along x march along y; 3D: 64 x 4 threads march along z): the rows or
// planes of v_1 sit in LDS, staged from the array w (LW) or evaluated
// from the fields once per staged point (c_1 psi_j (+ E_j)).  One slot
// (field); the two-slot launches and the launches without a Laplacian
// take fd_eq_kernel.
template <typename T, int DIM, int ST, bool LW, int NF, int HALO>
__global__ void __launch_bounds__(256) fd_eq_march_kernel(FDArgs a, FDEq q) {
  constexpr int BX = DIM == 2 ? FD2_BX : FD3_BX, BY = DIM == 2 ? 1 : FD3_BY;
  constexpr int RY = DIM == 2 ? 1 : fd3_rows(ST), TY = BY * RY;   // a thread's rows ty + BY r
  constexpr int NZ = DIM == 2 ? FD2_YC : FD3_ZC;            // planes a block marches
  constexpr int W = BX + 2 * HALO, H = DIM == 2 ? 1 : TY + 2 * HALO, NP = 2 * HALO + 1;
  constexpr int NV = (H * W + 255) / 256;
  __shared__ T pl[NP][H][W];
  const FDEqTab* tb = &q.tab;
  const int tid = threadIdx.x, tx = tid % BX, ty = tid / BX;
  const int64_t nbx = a.nx / BX, nby = DIM == 2 ? 1 : a.ny / TY;
  int64_t b = blockIdx.x;
  const int64_t bx = b % nbx;
  b /= nbx;
  const int64_t by = DIM == 2 ? 0 : b % nby, bm = DIM == 2 ? b : b / nby;
  const int64_t x0 = bx * BX, y0 = by * TY, m0 = bm * NZ;    // m: y in 2D, z in 3D
  const int64_t mx = a.nx - 1, my = a.ny - 1, mz = a.nz - 1;
  const T* f0 = (const T*)a.in[0];
  const T* f1 = NF == 2 ? (const T*)a.in[1] : f0;
  const int j = q.j[0];
  const T* fj = j == 0 ? f0 : f1;
  const T* w = (const T*)q.w[0];
  T* out = (T*)q.out[0];
  const T cl0 = (T)q.cl[0][0], cl1 = (T)q.cl[0][1];
  const int el0 = q.el[0][0], el1 = q.el[0][1];
  auto addr = [&](int p, int64_t m) -> int64_t {
    const int ly = p / W, lx = p - ly * W;
    const int64_t gx = (x0 + lx - HALO) & mx;
    if constexpr (DIM == 2) return ((m & my) << a.lx) + gx;
    else return (((m & mz) * a.ny + ((y0 + ly - HALO) & my)) << a.lx) + gx;
  };
  T n0[NV], n1[NV];
  auto fetch = [&](int64_t m) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int p = tid + 256 * v;
      if (p < H * W) {
        const int64_t g = addr(p, m);
        if constexpr (LW) {
          n0[v] = w[g];
        } else {
          n0[v] = f0[g];
          n1[v] = NF == 2 ? f1[g] : (T)0;
        }
      }
    }
  };
  auto store = [&](int slot) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int p = tid + 256 * v;
      if (p < H * W) {
        const int ly = p / W, lx = p - ly * W;
        T val;
        if constexpr (LW) {
          val = n0[v];
        } else {
          val = cl1 * (NF == 1 || j == 0 ? n0[v] : n1[v]);
          if (el1) val += fd_eq_E<T>(tb, j, n0[v], n1[v]);
        }
        pl[slot][ly][lx] = val;
      }
    }
  };
  // plane m + d of iteration k sits in slot (k + HALO + d) % NP
  for (int jj = 0; jj < 2 * HALO; ++jj) {
    fetch(m0 - HALO + jj);
    store(jj);
  }
  fetch(m0 + HALO);
  for (int k = 0; k < NZ; ++k) {
    const int64_t m = m0 + k;
    int64_t i[RY];
    T u[RY], uv[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      i[r] = DIM == 2 ? ((m << a.lx) + x0 + tid) : ((((m * a.ny) + y0 + ty + BY * r) << a.lx) + x0 + tx);
      u[r] = f0[i[r]];
      uv[r] = NF == 2 ? f1[i[r]] : (T)0;
    }
    store((k + 2 * HALO) % NP);
    if (k + 1 < NZ) fetch(m + HALO + 1);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int yl = ty + BY * r + HALO;
      auto at = [&](int64_t dx, int64_t dy, int64_t dz) -> T {
        if constexpr (DIM == 2) return pl[(k + HALO + (int)dy) % NP][0][tid + HALO + dx];
        else return pl[(k + HALO + (int)dz) % NP][yl + dy][tx + HALO + dx];
      };
      const T self = NF == 1 || j == 0 ? u[r] : uv[r];
      T v = cl0 * self + fd_stencil<T, DIM, ST>(at, a);
      if (el0) v += fd_eq_E<T>(tb, j, u[r], uv[r]);
      if (q.fin) v = self + (T)a.dt * v;
      out[i[r]] = v;
    }
    __syncthreads();   // the next iteration overwrites the plane m - HALO
  }
}

}  // namespace ss
