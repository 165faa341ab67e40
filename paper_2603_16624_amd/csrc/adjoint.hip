// Hand-written adjoint of (mover ->) moment gather for L = <gJ, J> + <gM, M>.
//
// One thread per particle recomputes the forward (stencils, gathers, alpha,
// velocity and position update) with the same device routines as the forward
// kernels, then runs the chain rule backwards:
//   moments:  dL/dvhat = (q/V) sum_a W'_a gJ[n'_a];  dL/dalpha' from gM over
//             the 36 stored corner pairs and from vhat = alpha' v';
//   rotation: dL/dB'_p by the vector-Jacobian product of Eq. 2;
//   weights:  dL/dxi' from dL/dW'_a, dL/dx' = dL/dxi' / h;
//   mover:    x' = x + dt v', v' = 2 alpha u - v, u = v + beta E_p (Eqs. 4-5, 8).
// Grid gradients gE, gB are scattered with atomics, summed first over the
// runs of lanes that share a node.
#include <algorithm>

#include "internal.h"

namespace ecsim {

namespace {

constexpr int kBlock = 256;
// The list kernel's few wavefronts are latency-bound (dependent gathers, then
// 72 scattered atomics per particle): one wavefront per workgroup spreads them
// over all compute units.
constexpr int kListBlock = 64;

// Adds v[0..NC) of every lane to dst[c][key] (key < 0: nothing). Lanes with
// equal keys in a contiguous run of the wavefront (cell-sorted particles
// share their corner nodes) are summed first, by a scan bounded by the run's
// first lane, and the run's last lane issues the atomics; a key that comes
// back in a later run is simply a run of its own. Reached by the whole
// wavefront.
template <typename T, int NC>
__device__ __forceinline__ void wave_run_add(int key, T (&v)[NC], T* const (&dst)[NC], int lane) {
  const int kprev = __shfl_up(key, 1);
  const bool head = lane == 0 || kprev != key;
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = heads & ((2ull << lane) - 1ull);   // heads at lanes <= lane
  const int start = 63 - __clzll(upto);
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const T o = __shfl_up(v[c], off);
      if (lane - off >= start) v[c] += o;
    }
  }
  const bool tail = lane == 63 || ((heads >> (lane + 1)) & 1ull);
  if (tail && key >= 0) {
#pragma unroll
    for (int c = 0; c < NC; ++c) unsafeAtomicAdd(dst[c] + key, v[c]);
  }
}

// Everything the adjoint of one species reads and writes.
template <typename T>
struct BwdArgs {
  Grid g;
  int np;
  const T *p0, *p1, *p2;
  const int32_t* cell;
  const T *v0, *v1, *v2;
  const T* q;
  T q_const, beta, dth0, dth1, dth2;
  T inv_V, beta_V;             // 1 / V and beta / V (cell volume V)
  T inv_h[3];                  // 1 / h per dimension
  const T *E, *B, *gJ, *gM;
  T *gx0, *gx1, *gx2, *gv0, *gv1, *gv2;
  T *gE, *gB;
  bool offset_grad;
  const int32_t* cell_start;   // cell ranges of the particles, or NULL
  int* nlist;                  // tiled kernel: count of the particles it leaves to the general path
  int* list;                   // ... and their indices
  T* gtab;                     // ... and every cell's table (kGS values per cell)
};

// The adjoint of particle p with every grid value read from memory (any
// order). Reached by the whole wavefront (the gradient scatter works across
// it); a lane with valid false recomputes particle p and stores nothing.
template <typename T, bool CELL, bool THROUGH>
__device__ __forceinline__ void backward_particle(const BwdArgs<T>& A, int p, bool valid, int lane) {
  const Grid& g = A.g;
  const T *const p0 = A.p0, *const p1 = A.p1, *const p2 = A.p2, *const v0 = A.v0, *const v1 = A.v1, *const v2 = A.v2;
  const int32_t* const cell = A.cell;
  const T* const q = A.q;
  const T q_const = A.q_const, beta = A.beta, dth0 = A.dth0, dth1 = A.dth1, dth2 = A.dth2;
  const T *const E = A.E, *const B = A.B, *const gJ = A.gJ, *const gM = A.gM;
  T *const gx0 = A.gx0, *const gx1 = A.gx1, *const gx2 = A.gx2, *const gv0 = A.gv0, *const gv1 = A.gv1,
    *const gv2 = A.gv2, *const gE = A.gE, *const gB = A.gB;
  const bool offset_grad = A.offset_grad;
  const int64_t nn = g.nn;
  const T qp = q ? q[p] : q_const;
  const T V = T(g.V);
  const T cj = qp / V;
  const T cm = (qp * beta) / V;
  const T h[3] = {T(g.hx), T(g.hy), T(g.hz)};

  Stencil<T> s0;
  if constexpr (CELL)
    s0 = stencil_cell(g, cell[p], p0[p], p1[p], p2[p]);
  else
    s0 = stencil_abs(g, p0[p], p1[p], p2[p]);
  Vec3<T> v{v0[p], v1[p], v2[p]};

  // ---- forward recompute ----
  T W0[8];
  int64_t nd0[8];
  T a0[9];
  Vec3<T> Bp{}, u{}, vn = v;
  Stencil<T> s1 = s0;
  if constexpr (THROUGH) {
    corners(g, s0, W0, nd0);
    Vec3<T> Ep = gather(E, nn, W0, nd0);
    Bp = gather(B, nn, W0, nd0);
    rotation(Bp, beta, a0);
    // alpha and u for the chain rule; the new velocity as the forward mover
    // computes it (so the recomputed push lands where the forward's did)
    velocity_update(a0, v, Ep, beta, u);
    vn = advance_velocity(Bp, beta, v, Ep);
    if constexpr (CELL) {
      int ix = s0.i[0], iy = s0.i[1], iz = s0.i[2];
      float ox = push_offset(s0.w1[0], vn.x, dth0, ix, g.nx);
      float oy = push_offset(s0.w1[1], vn.y, dth1, iy, g.ny);
      float oz = push_offset(s0.w1[2], vn.z, dth2, iz, g.nz);
      s1 = stencil_cell(g, ix + g.nx * (iy + g.ny * iz), ox, oy, oz);
    } else {
      s1 = stencil_abs(g, push_abs(p0[p], g.pdt[0], vn.x, g.nx * g.hx), push_abs(p1[p], g.pdt[1], vn.y, g.ny * g.hy),
                       push_abs(p2[p], g.pdt[2], vn.z, g.nz * g.hz));
    }
  }
  T W1[8];
  int64_t nd1[8];
  corners(g, s1, W1, nd1);
  Vec3<T> B1 = gather(B, nn, W1, nd1);
  T a1[9];
  rotation(B1, beta, a1);
  Vec3<T> vh = matvec(a1, vn);

  // ---- backward through the moments ----
  T gW1[8];
  Vec3<T> gvh{T(0), T(0), T(0)};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    T jx = gJ[nd1[c]], jy = gJ[nn + nd1[c]], jz = gJ[2 * nn + nd1[c]];
    T cw = cj * W1[c];
    gvh.x += cw * jx;
    gvh.y += cw * jy;
    gvh.z += cw * jz;
    gW1[c] = cj * ((jx * vh.x + jy * vh.y) + jz * vh.z);
  }
  T ga1[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) ga1[i] = T(0);
  // one corner a per step: its pairs' loads in flight together, without the
  // register pressure of all 36 pairs at once
#pragma unroll 1
  for (int ca = 0; ca < 8; ++ca) {
#pragma unroll
    for (int cb = ca; cb < 8; ++cb) {
      bool at_a;
      int k = pair_block(ca, cb, at_a);
      int64_t node = at_a ? nd1[ca] : nd1[cb];
      const T* G = gM + (int64_t)k * 9 * nn + node;
      T Gv[9];
      T sdot = T(0);
#pragma unroll
      for (int ij = 0; ij < 9; ++ij) {
        Gv[ij] = G[ij * nn];
        sdot += Gv[ij] * a1[ij];
      }
      T t = (cm * W1[ca]) * W1[cb];
#pragma unroll
      for (int ij = 0; ij < 9; ++ij) ga1[ij] += t * Gv[ij];
      if (ca == cb) {
        gW1[ca] += T(2) * cm * W1[ca] * sdot;
      } else {
        gW1[ca] += cm * W1[cb] * sdot;
        gW1[cb] += cm * W1[ca] * sdot;
      }
    }
  }
  // vhat = alpha' v'
  const T vv[3] = {vn.x, vn.y, vn.z};
  const T gh[3] = {gvh.x, gvh.y, gvh.z};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) ga1[3 * i + j] += gh[i] * vv[j];
  Vec3<T> gvn{(a1[0] * gh[0] + a1[3] * gh[1]) + a1[6] * gh[2], (a1[1] * gh[0] + a1[4] * gh[1]) + a1[7] * gh[2],
              (a1[2] * gh[0] + a1[5] * gh[1]) + a1[8] * gh[2]};
  // alpha' = R(B'_p), B'_p = sum W'_a B[n'_a]
  Vec3<T> gB1 = rotation_vjp(a1, B1, beta, ga1);
  T* const dstB[3] = {gB, gB + nn, gB + 2 * nn};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    T v3[3] = {valid ? W1[c] * gB1.x : T(0), valid ? W1[c] * gB1.y : T(0), valid ? W1[c] * gB1.z : T(0)};
    wave_run_add<T, 3>(valid ? (int)nd1[c] : -1, v3, dstB, lane);
    gW1[c] += (B[nd1[c]] * gB1.x + B[nn + nd1[c]] * gB1.y) + B[2 * nn + nd1[c]] * gB1.z;
  }
  T gxi1[3];
  weight_grad(s1, gW1, gxi1);
  Vec3<T> gx{gxi1[0] / h[0], gxi1[1] / h[1], gxi1[2] / h[2]};
  Vec3<T> gv = gvn;

  if constexpr (THROUGH) {
    // x' = x + dt v' (wrap is a constant shift; no push along a dimension of
    // one cell)
    gvn.x += T(g.pdt[0]) * gx.x;
    gvn.y += T(g.pdt[1]) * gx.y;
    gvn.z += T(g.pdt[2]) * gx.z;
    // v' = 2 vbar - v, vbar = alpha u
    Vec3<T> gvb{T(2) * gvn.x, T(2) * gvn.y, T(2) * gvn.z};
    gv = Vec3<T>{-gvn.x, -gvn.y, -gvn.z};
    const T uu[3] = {u.x, u.y, u.z};
    const T gb[3] = {gvb.x, gvb.y, gvb.z};
    T ga0[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) ga0[3 * i + j] = gb[i] * uu[j];
    Vec3<T> gu{(a0[0] * gb[0] + a0[3] * gb[1]) + a0[6] * gb[2], (a0[1] * gb[0] + a0[4] * gb[1]) + a0[7] * gb[2],
               (a0[2] * gb[0] + a0[5] * gb[1]) + a0[8] * gb[2]};
    // u = v + beta E_p
    gv.x += gu.x;
    gv.y += gu.y;
    gv.z += gu.z;
    Vec3<T> gEp{beta * gu.x, beta * gu.y, beta * gu.z};
    Vec3<T> gBp = rotation_vjp(a0, Bp, beta, ga0);
    T gW0[8];
    T* const dstEB[6] = {gE, gE + nn, gE + 2 * nn, gB, gB + nn, gB + 2 * nn};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      T v6[6] = {W0[c] * gEp.x, W0[c] * gEp.y, W0[c] * gEp.z, W0[c] * gBp.x, W0[c] * gBp.y, W0[c] * gBp.z};
#pragma unroll
      for (int k = 0; k < 6; ++k) v6[k] = valid ? v6[k] : T(0);
      wave_run_add<T, 6>(valid ? (int)nd0[c] : -1, v6, dstEB, lane);
      gW0[c] = ((E[nd0[c]] * gEp.x + E[nn + nd0[c]] * gEp.y) + E[2 * nn + nd0[c]] * gEp.z) +
               ((B[nd0[c]] * gBp.x + B[nn + nd0[c]] * gBp.y) + B[2 * nn + nd0[c]] * gBp.z);
    }
    T gxi0[3];
    weight_grad(s0, gW0, gxi0);
    gx.x += gxi0[0] / h[0];
    gx.y += gxi0[1] / h[1];
    gx.z += gxi0[2] / h[2];
  }
  if (offset_grad) {   // FP32 form: d/d(offset) = h d/dx
    gx.x *= h[0];
    gx.y *= h[1];
    gx.z *= h[2];
  }
  note_nonfinite(g, valid && !(finite(gx.x) && finite(gx.y) && finite(gx.z) && finite(gv.x) && finite(gv.y) &&
                               finite(gv.z)));
  if (valid) {
    gx0[p] = gx.x;
    gx1[p] = gx.y;
    gx2[p] = gx.z;
    gv0[p] = gv.x;
    gv1[p] = gv.y;
    gv2[p] = gv.z;
  }
}

// any order: one thread per particle; lanes past the end recompute the last
// particle and store nothing
template <typename T, bool CELL, bool THROUGH>
__global__ void __launch_bounds__(kBlock) k_backward(BwdArgs<T> A) {
  const int lane = threadIdx.x & 63;
  const bool valid = blockIdx.x * kBlock + threadIdx.x < A.np;
  const int p = valid ? blockIdx.x * kBlock + threadIdx.x : A.np - 1;
  backward_particle<T, CELL, THROUGH>(A, p, valid, lane);
}

// ---------------------------------------------------------------------------
// brick-tiled adjoint (particles grouped by cell) and the per-cell tables
// ---------------------------------------------------------------------------
// For a particle whose moments fall in cell c (its post-move cell), every
// value of gJ and gM its adjoint reads belongs to c: gJ at the 8 corners and
// gM over the cell's 36 stored corner pairs. Since the weight product of pair
// (a, b) depends on the class a + b only, the moment part of its loss is
//   l = (q/V) (alpha' v') . sum_a W'_a gJ_a + (q beta/V) sum_c m_c(xi') <G_c, alpha'>,
// with G_c the sum of gM over the cell's pairs of class c (27 blocks of 9).
// The table of cell c holds G_c and gJ at its corners: kGS values, G first.
constexpr int kGS = 268;   // 27 x 9 + 8 x 3 + 1 pad (16-byte rows in FP32 and FP64)
// In LDS the tables sit kGL apart: an odd stride puts the same value of the
// wavefront's 8 cells (local cells 4 apart) in distinct banks.
constexpr int kGL = 269;

// The grid-gradient sources of one particle: pre-move corners a take
// W0_a gE_p and W0_a gB_p, post-move corners W1_a gB'_p (W1 from the
// post-move stencil s1).
template <typename T>
struct GridSrc {
  Stencil<T> s1;
  Vec3<T> gEp, gBp, gB1;
};

// The adjoint of one particle from its pre-move stencil s0, velocity v and
// charge qp. pre(a, k): value k (E x, y, z, then B x, y, z) at pre-move
// corner a. post_of(s1, c1): the post-move cell's accessor, with B(a, k) at
// its corner a (k = 0..2) and G, its table (FROM_MEMORY: in global memory,
// else in LDS). Returns the particle's gradients
// (position gradient per unit length) and its grid-gradient sources; c1 is
// the post-move cell.
template <typename T, bool CELL, bool THROUGH, bool FROM_MEMORY, class Pre, class PostOf>
__device__ __forceinline__ void adjoint_core(const BwdArgs<T>& A, const Stencil<T>& s0, T xa, T xb, T xc, Vec3<T> v,
                                             T qp, Pre pre, PostOf post_of, Vec3<T>& gx, Vec3<T>& gv,
                                             GridSrc<T>& src, int& c1) {
  const Grid& g = A.g;
  // ---- forward recompute ----
  T W0[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) W0[a] = corner_weight(s0, a);
  T a0[9];
  Vec3<T> Bp{T(0), T(0), T(0)}, Ep{T(0), T(0), T(0)}, u{T(0), T(0), T(0)}, vn = v;
  Stencil<T> s1 = s0;
  if constexpr (THROUGH) {
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      Ep.x = fma(W0[a], pre(a, 0), Ep.x);
      Ep.y = fma(W0[a], pre(a, 1), Ep.y);
      Ep.z = fma(W0[a], pre(a, 2), Ep.z);
      Bp.x = fma(W0[a], pre(a, 3), Bp.x);
      Bp.y = fma(W0[a], pre(a, 4), Bp.y);
      Bp.z = fma(W0[a], pre(a, 5), Bp.z);
    }
    rotation(Bp, A.beta, a0);
    // alpha and u for the chain rule; the new velocity as the forward mover
    // computes it (so the recomputed push lands where the forward's did)
    velocity_update(a0, v, Ep, A.beta, u);
    vn = advance_velocity(Bp, A.beta, v, Ep);
    if constexpr (CELL) {
      int ix = s0.i[0], iy = s0.i[1], iz = s0.i[2];
      const float ox = push_offset(s0.w1[0], vn.x, A.dth0, ix, g.nx);
      const float oy = push_offset(s0.w1[1], vn.y, A.dth1, iy, g.ny);
      const float oz = push_offset(s0.w1[2], vn.z, A.dth2, iz, g.nz);
      s1 = stencil_cell(g, ix + g.nx * (iy + g.ny * iz), ox, oy, oz);
    } else {
      s1 = stencil_abs(g, push_abs(xa, g.pdt[0], vn.x, g.nx * g.hx), push_abs(xb, g.pdt[1], vn.y, g.ny * g.hy),
                       push_abs(xc, g.pdt[2], vn.z, g.nz * g.hz));
    }
  }
  c1 = s1.i[0] + g.nx * (s1.i[1] + g.ny * s1.i[2]);
  src.s1 = s1;
  const auto post = post_of(s1, c1);
  // ---- moments at the post-move state ----
  const T cj = qp * A.inv_V;
  const T cm = qp * A.beta_V;
  T W1[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) W1[a] = corner_weight(s1, a);
  Vec3<T> B1{T(0), T(0), T(0)};
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    B1.x = fma(W1[a], post.B(a, 0), B1.x);
    B1.y = fma(W1[a], post.B(a, 1), B1.y);
    B1.z = fma(W1[a], post.B(a, 2), B1.z);
  }
  T a1[9];
  rotation(B1, A.beta, a1);
  const Vec3<T> vh = matvec(a1, vn);
  // from LDS the corner fields are read again below rather than held in
  // registers
  if constexpr (!FROM_MEMORY) asm volatile("" ::: "memory");
  const T* const G = post.G;
  // J part: dL/dvhat and dL/dW'_a
  T gW1[8];
  Vec3<T> gvh{T(0), T(0), T(0)};
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const T jx = G[243 + 3 * a], jy = G[244 + 3 * a], jz = G[245 + 3 * a];
    const T cw = cj * W1[a];
    gvh.x += cw * jx;
    gvh.y += cw * jy;
    gvh.z += cw * jz;
    gW1[a] = cj * ((jx * vh.x + jy * vh.y) + jz * vh.z);
  }
  // M part: dL/dalpha' = (q beta/V) sum_c m_c G_c; dL/dm_c = (q beta/V) <G_c, alpha'>
  T f[3][3], df[3][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const T w0 = s1.w0[d], w1 = s1.w1[d];
    f[d][0] = w0 * w0;
    f[d][1] = w0 * w1;
    f[d][2] = w1 * w1;
    df[d][0] = T(-2) * w0;
    df[d][1] = w0 - w1;
    df[d][2] = T(2) * w1;
  }
  // classes c = cx + 3 cy + 9 cz, weight m_c = f_x[cx] f_y[cy] f_z[cz]
  T H[9];
#pragma unroll
  for (int ij = 0; ij < 9; ++ij) H[ij] = T(0);
  T gxi1[3] = {T(0), T(0), T(0)};
  // one row (cy, cz) of three classes per step
  auto class_row = [&](int row) {
    const int cy = row % 3, cz = row / 3;
    const T fy = cy == 0 ? f[1][0] : (cy == 1 ? f[1][1] : f[1][2]);
    const T dy = cy == 0 ? df[1][0] : (cy == 1 ? df[1][1] : df[1][2]);
    const T fz = cz == 0 ? f[2][0] : (cz == 1 ? f[2][1] : f[2][2]);
    const T dz = cz == 0 ? df[2][0] : (cz == 1 ? df[2][1] : df[2][2]);
#pragma unroll
    for (int cx = 0; cx < 3; ++cx) {
      const T* const Gc = G + (cx + 3 * row) * 9;
      const T mxy = f[0][cx] * fy;
      const T m = mxy * fz;
      T D = T(0);
#pragma unroll
      for (int ij = 0; ij < 9; ++ij) {
        const T Gv = Gc[ij];
        H[ij] = fma(m, Gv, H[ij]);
        D = fma(Gv, a1[ij], D);
      }
      gxi1[0] = fma(D, (df[0][cx] * fy) * fz, gxi1[0]);
      gxi1[1] = fma(D, (f[0][cx] * dy) * fz, gxi1[1]);
      gxi1[2] = fma(D, mxy * dz, gxi1[2]);
    }
  };
  if constexpr (FROM_MEMORY) {
    // the table in global memory: every load issued up front
#pragma unroll
    for (int row = 0; row < 9; ++row) class_row(row);
  } else {
    // the table in LDS: a rolled loop keeps the registers for occupancy
#pragma unroll 1
    for (int row = 0; row < 9; ++row) class_row(row);
  }
  T ga1[9];
  const T vv[3] = {vn.x, vn.y, vn.z};
  const T gh[3] = {gvh.x, gvh.y, gvh.z};
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) ga1[3 * r + cc] = fma(cm, H[3 * r + cc], gh[r] * vv[cc]);
  Vec3<T> gvn{(a1[0] * gh[0] + a1[3] * gh[1]) + a1[6] * gh[2], (a1[1] * gh[0] + a1[4] * gh[1]) + a1[7] * gh[2],
              (a1[2] * gh[0] + a1[5] * gh[1]) + a1[8] * gh[2]};
  // alpha' = R(B'_p), B'_p = sum W'_a B_a
  src.gB1 = rotation_vjp(a1, B1, A.beta, ga1);
#pragma unroll
  for (int a = 0; a < 8; ++a) gW1[a] += (post.B(a, 0) * src.gB1.x + post.B(a, 1) * src.gB1.y) + post.B(a, 2) * src.gB1.z;
  T gxiw[3];
  weight_grad(s1, gW1, gxiw);
  // gradients with respect to the offsets xi (d/dx = (1/h) d/dxi)
  T go[3] = {fma(cm, gxi1[0], gxiw[0]), fma(cm, gxi1[1], gxiw[1]), fma(cm, gxi1[2], gxiw[2])};
  gv = gvn;
  src.gEp = Vec3<T>{T(0), T(0), T(0)};
  src.gBp = Vec3<T>{T(0), T(0), T(0)};
  if constexpr (THROUGH) {
    // x' = x + dt v', i.e. xi' = xi + (dt / h) v' (no push along a dimension
    // of one cell)
    gvn.x = fma(A.dth0, go[0], gvn.x);
    gvn.y = fma(A.dth1, go[1], gvn.y);
    gvn.z = fma(A.dth2, go[2], gvn.z);
    // v' = 2 vbar - v, vbar = alpha u, u = v + beta E_p
    const Vec3<T> gvb{T(2) * gvn.x, T(2) * gvn.y, T(2) * gvn.z};
    gv = Vec3<T>{-gvn.x, -gvn.y, -gvn.z};
    const T uu[3] = {u.x, u.y, u.z};
    const T gb[3] = {gvb.x, gvb.y, gvb.z};
    T ga0[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) ga0[3 * r + cc] = gb[r] * uu[cc];
    const Vec3<T> gu{(a0[0] * gb[0] + a0[3] * gb[1]) + a0[6] * gb[2], (a0[1] * gb[0] + a0[4] * gb[1]) + a0[7] * gb[2],
                     (a0[2] * gb[0] + a0[5] * gb[1]) + a0[8] * gb[2]};
    gv.x += gu.x;
    gv.y += gu.y;
    gv.z += gu.z;
    src.gEp = Vec3<T>{A.beta * gu.x, A.beta * gu.y, A.beta * gu.z};
    src.gBp = rotation_vjp(a0, Bp, A.beta, ga0);
    T gW0[8];
#pragma unroll
    for (int a = 0; a < 8; ++a)
      gW0[a] = ((pre(a, 0) * src.gEp.x + pre(a, 1) * src.gEp.y) + pre(a, 2) * src.gEp.z) +
               ((pre(a, 3) * src.gBp.x + pre(a, 4) * src.gBp.y) + pre(a, 5) * src.gBp.z);
    T gxi0[3];
    weight_grad(s0, gW0, gxi0);
    go[0] += gxi0[0];
    go[1] += gxi0[1];
    go[2] += gxi0[2];
  }
  if (A.offset_grad) gx = Vec3<T>{go[0], go[1], go[2]};   // FP32 form: d/d(offset)
  else gx = Vec3<T>{go[0] * A.inv_h[0], go[1] * A.inv_h[1], go[2] * A.inv_h[2]};
}

// Per-cell tables of one brick: item (value ij, cell) sums gM over the cell's
// pairs of each class; the last item per cell copies gJ at its corners.
template <typename T, int TX, int TY, int TZ, class NodeOf>
__device__ __forceinline__ void form_tables(const BwdArgs<T>& A, NodeOf node_of, T* cg, int tid, int nthreads) {
  constexpr int NCELL = TX * TY * TZ;
  const int64_t nn = A.g.nn;
  for (int it = tid; it < NCELL * 10; it += nthreads) {
    const int ij = it / NCELL, lc = it % NCELL;
    const int lx = lc % TX, ly = (lc / TX) % TY, lz = lc / (TX * TY);
    T* const G = cg + lc * kGL;
    if (ij < 9) {
      T Gc[27];
#pragma unroll
      for (int c = 0; c < 27; ++c) Gc[c] = T(0);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
#pragma unroll
        for (int b = a; b < 8; ++b) {
          bool at_a;
          const int k = pair_block(a, b, at_a);
          const int t = at_a ? a : b;
          const int64_t node = node_of(lx + (t & 1), ly + ((t >> 1) & 1), lz + ((t >> 2) & 1));
          const int cls = ((a & 1) + (b & 1)) + 3 * (((a >> 1) & 1) + ((b >> 1) & 1)) +
                          9 * (((a >> 2) & 1) + ((b >> 2) & 1));
          Gc[cls] += A.gM[(int64_t)(k * 9 + ij) * nn + node];
        }
      }
#pragma unroll
      for (int c = 0; c < 27; ++c) G[c * 9 + ij] = Gc[c];
    } else {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int64_t node = node_of(lx + (a & 1), ly + ((a >> 1) & 1), lz + ((a >> 2) & 1));
#pragma unroll
        for (int c = 0; c < 3; ++c) G[243 + 3 * a + c] = A.gJ[c * nn + node];
      }
      G[kGS - 1] = T(0);
    }
  }
}

// The particles the tiled kernel listed (not in their range's cell before
// the move, or outside it after): one lane per entry, fields and gradients in
// memory, the post-move cell's table from the tiled kernel's copy of every
// cell's table, plain atomics for the grid gradients (the listed particles
// are scattered).
template <typename T, bool CELL, bool THROUGH>
__global__ void __launch_bounds__(kListBlock) k_backward_list(BwdArgs<T> A) {
  const Grid& g = A.g;
  const int64_t nn = g.nn;
  const int n = *A.nlist;
  for (int base = blockIdx.x * kListBlock; base < n; base += gridDim.x * kListBlock) {
    const int i = base + (int)threadIdx.x;
    if (i >= n) break;
    const int p = A.list[i];
    Stencil<T> s0;
    if constexpr (CELL) s0 = stencil_cell(g, A.cell[p], A.p0[p], A.p1[p], A.p2[p]);
    else s0 = stencil_abs(g, A.p0[p], A.p1[p], A.p2[p]);
    const Vec3<T> v{A.v0[p], A.v1[p], A.v2[p]};
    const T qp = A.q ? A.q[p] : A.q_const;
    int64_t nd0[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) nd0[a] = corner_node(g, s0, a);
    auto pre = [&](int a, int k) -> T { return (k < 3 ? A.E : A.B)[(int64_t)(k % 3) * nn + nd0[a]]; };
    int64_t nd1[8];
    auto post_of = [&](const Stencil<T>& s1, int c1) {
#pragma unroll
      for (int a = 0; a < 8; ++a) nd1[a] = corner_node(g, s1, a);
      struct Post {
        const T* Bf;
        const int64_t* nd;
        int64_t nn;
        const T* G;
        __device__ T B(int a, int k) const { return Bf[(int64_t)k * nn + nd[a]]; }
      };
      return Post{A.B, nd1, nn, A.gtab + (int64_t)c1 * kGS};
    };
    Vec3<T> gx, gv;
    GridSrc<T> src;
    int c1;
    adjoint_core<T, CELL, THROUGH, true>(A, s0, A.p0[p], A.p1[p], A.p2[p], v, qp, pre, post_of, gx, gv, src, c1);
    note_nonfinite(g, !(finite(gx.x) && finite(gx.y) && finite(gx.z) && finite(gv.x) && finite(gv.y) &&
                        finite(gv.z)));
    A.gx0[p] = gx.x;
    A.gx1[p] = gx.y;
    A.gx2[p] = gx.z;
    A.gv0[p] = gv.x;
    A.gv1[p] = gv.y;
    A.gv2[p] = gv.z;
    const T gb1[3] = {src.gB1.x, src.gB1.y, src.gB1.z};
    const T gep[3] = {src.gEp.x, src.gEp.y, src.gEp.z};
    const T gbp[3] = {src.gBp.x, src.gBp.y, src.gBp.z};
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const T w0 = corner_weight(s0, a), w1 = corner_weight(src.s1, a);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        unsafeAtomicAdd(A.gB + (int64_t)k * nn + nd1[a], w1 * gb1[k]);
        if constexpr (THROUGH) {
          unsafeAtomicAdd(A.gE + (int64_t)k * nn + nd0[a], w0 * gep[k]);
          unsafeAtomicAdd(A.gB + (int64_t)k * nn + nd0[a], w0 * gbp[k]);
        }
      }
    }
  }
}

// A workgroup owns a brick of cells: it stages E and B at the brick's nodes
// and forms its cells' tables in LDS (and writes them to the workspace's copy,
// which the listed particles read). Each wavefront takes cells wave + NW j of
// the brick and gives each of them ceil(n_j / C) lanes, with C the least
// count per lane for which they fit the wavefront; the lanes of a cell take
// its particles in turn (consecutive lanes, consecutive particles), so each
// lane meets one cell only and sums its grid-gradient sources at that cell's
// 8 corners in registers. After the wavefront's last step the lanes of each
// cell are summed (a tree within the cell's lanes) and added to per-node sums
// in LDS, which go to gE and gB with one atomic per node value at the end
// (adding every particle's sources to LDS directly, 48 atomics per particle
// on the few addresses of a cell, measured twice as slow). A
// particle that is not in its range's cell before the move, or leaves it in
// the move, is listed for k_backward_list and contributes nothing here.
template <typename T, int TX, int TY, int TZ, int NW, bool THROUGH>
__global__ void __launch_bounds__(NW * 64) k_backward_tiled(BwdArgs<T> A, int ntx, int nty, int ntz) {
  constexpr bool CELL = sizeof(T) == 4;
  constexpr int NCELL = TX * TY * TZ;
  constexpr int CPW = NCELL / NW;   // cells per wavefront
  static_assert(NCELL % NW == 0 && CPW <= 32 && (CPW & (CPW - 1)) == 0, "a power-of-two cell count per wavefront");
  constexpr int NX = TX + 1, NY = TY + 1, NZ = TZ + 1, NBN = NX * NY * NZ;
  __shared__ __attribute__((aligned(16))) T cg[NCELL * kGL];
  __shared__ __attribute__((aligned(16))) T nf[NBN * 8];   // per node: E (3), B (3), pad
  __shared__ T acc[NBN * 8];                              // per node: gE (3), gB (3), pad
  __shared__ int64_t bnode[NBN];                          // global index of each brick node
  const Grid& g = A.g;
  const int64_t nn = g.nn;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int x0, y0, z0;
  brick_origin<TX, TY, TZ>(ntx, nty, ntz, x0, y0, z0);

  for (int nl = tid; nl < NBN; nl += NW * 64) {
    const int gx = (x0 + nl % NX) % g.nx, gy = (y0 + (nl / NX) % NY) % g.ny, gz = (z0 + nl / (NX * NY)) % g.nz;
    bnode[nl] = gx + (int64_t)g.nx * (gy + (int64_t)g.ny * gz);
  }
  __syncthreads();
  auto node_of = [&](int lx, int ly, int lz) -> int64_t { return bnode[lx + NX * (ly + NY * lz)]; };
  for (int nl = tid; nl < NBN; nl += NW * 64) {
    const int64_t gn = bnode[nl];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      nf[8 * nl + c] = THROUGH ? A.E[c * nn + gn] : T(0);
      nf[8 * nl + 3 + c] = A.B[c * nn + gn];
      acc[8 * nl + c] = T(0);
      acc[8 * nl + 3 + c] = T(0);
    }
    nf[8 * nl + 6] = nf[8 * nl + 7] = T(0);
    acc[8 * nl + 6] = acc[8 * nl + 7] = T(0);
  }
  form_tables<T, TX, TY, TZ>(A, node_of, cg, tid, NW * 64);
  __syncthreads();
  // the copy of the tables for the listed particles (cells of the grid only)
  for (int it = tid; it < NCELL * kGS; it += NW * 64) {
    const int lc = it / kGS, e = it % kGS;
    const int cx = x0 + lc % TX, cy = y0 + (lc / TX) % TY, cz = z0 + lc / (TX * TY);
    if (cx < g.nx && cy < g.ny && cz < g.nz)
      A.gtab[(int64_t)(cx + g.nx * (cy + g.ny * cz)) * kGS + e] = cg[lc * kGL + e];
  }

  // ---- the wavefront's cells (lane j < CPW: local cell wave + NW j) ----
  int cnt = 0, beg = 0, gcell = -1;
  if (lane < CPW) {
    const int lc = wave + NW * lane;
    const int cx = x0 + lc % TX, cy = y0 + (lc / TX) % TY, cz = z0 + lc / (TX * TY);
    if (cx < g.nx && cy < g.ny && cz < g.nz) {
      gcell = cx + g.nx * (cy + g.ny * cz);
      beg = A.cell_start[gcell];
      cnt = A.cell_start[gcell + 1] - beg;
    }
  }
  int total = cnt;
#pragma unroll
  for (int o = 1; o < CPW; o <<= 1) total += __shfl_xor(total, o);
  total = __builtin_amdgcn_readfirstlane(total);
  // particles per lane: the least C with sum_j ceil(n_j / C) <= 64
  int C = total > 0 ? (total + 63) / 64 : 0;
  int m = 0;   // lanes of cell j (lane j < CPW)
  if (C > 0) {
    for (;;) {
      m = lane < CPW ? (cnt + C - 1) / C : 0;
      int sm = m;
#pragma unroll
      for (int o = 1; o < CPW; o <<= 1) sm += __shfl_xor(sm, o);
      if (__builtin_amdgcn_readfirstlane(sm) <= 64) break;
      ++C;
    }
  }
  int incl = m;
#pragma unroll
  for (int o = 1; o < CPW; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  // first lane of each cell and the lanes in use, in scalar registers
  int ofs[CPW + 1];
  ofs[0] = 0;
#pragma unroll
  for (int k = 0; k < CPW; ++k) ofs[k + 1] = __builtin_amdgcn_readlane(incl, k);
  int mmax = 0;
#pragma unroll
  for (int k = 0; k < CPW; ++k) mmax = max(mmax, ofs[k + 1] - ofs[k]);
  // this lane's cell j and its rank r among the cell's lanes
  int j = 0;
#pragma unroll
  for (int k = 1; k < CPW; ++k) j += lane >= ofs[k] ? 1 : 0;
  const bool own = lane < ofs[CPW];
  const int r = lane - __shfl(incl - m, j);
  const int mj = __shfl(m, j);
  const int nj = __shfl(cnt, j);
  const int bj = __shfl(beg, j);
  const int cj = __shfl(gcell, j);
  const int lc = wave + NW * j;
  const T* const nb = nf + 8 * ((lc % TX) + NX * ((lc / TX) % TY + NY * (lc / (TX * TY))));
  auto corner = [&](int a) -> const T* { return nb + 8 * ((a & 1) + NX * (((a >> 1) & 1) + NY * ((a >> 2) & 1))); };
  auto pre = [&](int a, int k) -> T { return corner(a)[k]; };
  const T* const Gcell = cg + lc * kGL;
  auto post_of = [&](const Stencil<T>&, int) {
    struct Post {
      const T* nb;
      const T* G;
      __device__ T B(int a, int k) const {
        return nb[8 * ((a & 1) + NX * (((a >> 1) & 1) + NY * ((a >> 2) & 1))) + 3 + k];
      }
    };
    return Post{nb, Gcell};
  };

  // grid-gradient sums at the cell's corners: [a][gE x, y, z, gB x, y, z]
  T sum[8][6];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int k = 0; k < 6; ++k) sum[a][k] = T(0);

  for (int step = 0; step < C; ++step) {
    const int i = r + step * mj;
    const bool valid = own && i < nj;
    const int p = valid ? bj + i : 0;
    Stencil<T> s0;
    if constexpr (CELL) s0 = stencil_cell(g, A.cell[p], A.p0[p], A.p1[p], A.p2[p]);
    else s0 = stencil_abs(g, A.p0[p], A.p1[p], A.p2[p]);
    const int c0 = s0.i[0] + g.nx * (s0.i[1] + g.ny * s0.i[2]);
    const Vec3<T> v{A.v0[p], A.v1[p], A.v2[p]};
    const T qp = A.q ? A.q[p] : A.q_const;
    Vec3<T> gx, gv;
    GridSrc<T> src;
    int c1;
    adjoint_core<T, CELL, THROUGH, false>(A, s0, A.p0[p], A.p1[p], A.p2[p], v, qp, pre, post_of, gx, gv, src, c1);
    const bool fast = valid && c0 == cj && c1 == cj;
    // the others go to the general path (a second kernel over the list)
    {
      const uint64_t mk = __ballot(valid && !fast);
      if (mk) {   // wave-uniform
        int b0 = 0;
        if (lane == 0) b0 = atomicAdd(A.nlist, __popcll(mk));
        b0 = __builtin_amdgcn_readfirstlane(b0);
        if (valid && !fast) A.list[b0 + __popcll(mk & ((1ull << lane) - 1ull))] = p;
      }
    }
    note_nonfinite(g, fast && !(finite(gx.x) && finite(gx.y) && finite(gx.z) && finite(gv.x) && finite(gv.y) &&
                                finite(gv.z)));
    if (fast) {
      A.gx0[p] = gx.x;
      A.gx1[p] = gx.y;
      A.gx2[p] = gx.z;
      A.gv0[p] = gv.x;
      A.gv1[p] = gv.y;
      A.gv2[p] = gv.z;
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const T w1 = corner_weight(src.s1, a);
        if constexpr (THROUGH) {
          const T w0 = corner_weight(s0, a);
          sum[a][0] = fma(w0, src.gEp.x, sum[a][0]);
          sum[a][1] = fma(w0, src.gEp.y, sum[a][1]);
          sum[a][2] = fma(w0, src.gEp.z, sum[a][2]);
          sum[a][3] = fma(w1, src.gB1.x, fma(w0, src.gBp.x, sum[a][3]));
          sum[a][4] = fma(w1, src.gB1.y, fma(w0, src.gBp.y, sum[a][4]));
          sum[a][5] = fma(w1, src.gB1.z, fma(w0, src.gBp.z, sum[a][5]));
        } else {
          sum[a][3] = fma(w1, src.gB1.x, sum[a][3]);
          sum[a][4] = fma(w1, src.gB1.y, sum[a][4]);
          sum[a][5] = fma(w1, src.gB1.z, sum[a][5]);
        }
      }
    }
  }
  // ---- the cell sums: a tree over each cell's lanes, then its first lane
  // adds them to the brick's node sums ----
  if (C > 0) {   // wave-uniform
    for (int off = 1; off < mmax; off <<= 1) {
      const bool take = r + off < mj;
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          if (!THROUGH && k < 3) continue;
          const T o = __shfl_down(sum[a][k], off);
          sum[a][k] += take ? o : T(0);
        }
    }
    if (own && r == 0) {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        T* const an = acc + (corner(a) - nf);
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (THROUGH || k >= 3) atomicAdd(an + k, sum[a][k]);
      }
    }
  }
  __syncthreads();
  // the brick's node sums to the global gradients (face nodes are shared
  // with the neighbouring bricks)
  for (int it = tid; it < NBN * 6; it += NW * 64) {
    const int nl = it / 6, k = it % 6;
    const T v = acc[8 * nl + k];
    if (v == T(0)) continue;
    const int64_t gn = bnode[nl];
    unsafeAtomicAdd((k < 3 ? A.gE : A.gB) + (int64_t)(k % 3) * nn + gn, v);
  }
}

}  // namespace

size_t backward_table_offset(int64_t np);

namespace {

template <typename T, bool CELL>
hipError_t launch_T(const Grid& g, const SpeciesArgs& sp, const void* E, const void* B, const void* gJ,
                    const void* gM, void* const gpos[3], void* const gvel[3], void* gE, void* gB, bool through,
                    bool offset_grad, void* ws, hipStream_t st) {
  BwdArgs<T> A;
  A.g = g;
  A.np = sp.np;
  A.p0 = (const T*)sp.pos[0];
  A.p1 = (const T*)sp.pos[1];
  A.p2 = (const T*)sp.pos[2];
  A.cell = sp.cell;
  A.v0 = (const T*)sp.vel[0];
  A.v1 = (const T*)sp.vel[1];
  A.v2 = (const T*)sp.vel[2];
  A.q = (const T*)sp.q;
  A.q_const = (T)sp.q_const;
  A.beta = (T)(sp.qom * g.dt / 2.0);
  A.inv_V = (T)(1.0 / g.V);
  A.beta_V = (T)(sp.qom * g.dt / 2.0 / g.V);
  A.inv_h[0] = (T)(1.0 / g.hx);
  A.inv_h[1] = (T)(1.0 / g.hy);
  A.inv_h[2] = (T)(1.0 / g.hz);
  A.dth0 = (T)(g.pdt[0] / g.hx);
  A.dth1 = (T)(g.pdt[1] / g.hy);
  A.dth2 = (T)(g.pdt[2] / g.hz);
  A.E = (const T*)E;
  A.B = (const T*)B;
  A.gJ = (const T*)gJ;
  A.gM = (const T*)gM;
  A.gx0 = (T*)gpos[0];
  A.gx1 = (T*)gpos[1];
  A.gx2 = (T*)gpos[2];
  A.gv0 = (T*)gvel[0];
  A.gv1 = (T*)gvel[1];
  A.gv2 = (T*)gvel[2];
  A.gE = (T*)gE;
  A.gB = (T*)gB;
  A.offset_grad = offset_grad;
  A.cell_start = sp.cell_start;
  if (sp.cell_start) {
    // particles grouped by cell: the brick-tiled kernel, then the particles
    // it listed; the workspace holds the list's count, the list and every
    // cell's table
    A.nlist = (int*)ws;
    A.list = (int*)((char*)ws + 256);
    A.gtab = (T*)((char*)ws + backward_table_offset(sp.np));
    hipError_t e = launch_zero(ws, 256, st);
    if (e != hipSuccess) return e;
    constexpr int NW = 4;
    if (g.nz == 1) {
      const int ntx = (g.nx + 7) / 8, nty = (g.ny + 3) / 4;
      if (through)
        hipLaunchKernelGGL((k_backward_tiled<T, 8, 4, 1, NW, true>), dim3(ntx * nty), dim3(NW * 64), 0, st, A, ntx,
                           nty, 1);
      else
        hipLaunchKernelGGL((k_backward_tiled<T, 8, 4, 1, NW, false>), dim3(ntx * nty), dim3(NW * 64), 0, st, A, ntx,
                           nty, 1);
    } else {
      const int ntx = (g.nx + 3) / 4, nty = (g.ny + 3) / 4, ntz = (g.nz + 1) / 2;
      if (through)
        hipLaunchKernelGGL((k_backward_tiled<T, 4, 4, 2, NW, true>), dim3(ntx * nty * ntz), dim3(NW * 64), 0, st, A,
                           ntx, nty, ntz);
      else
        hipLaunchKernelGGL((k_backward_tiled<T, 4, 4, 2, NW, false>), dim3(ntx * nty * ntz), dim3(NW * 64), 0, st, A,
                           ntx, nty, ntz);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const unsigned lb = (unsigned)std::min<int64_t>(4096, (sp.np + kListBlock - 1) / kListBlock);
    if (through)
      hipLaunchKernelGGL((k_backward_list<T, CELL, true>), dim3(lb), dim3(kListBlock), 0, st, A);
    else
      hipLaunchKernelGGL((k_backward_list<T, CELL, false>), dim3(lb), dim3(kListBlock), 0, st, A);
    return hipGetLastError();
  }
  dim3 grid((unsigned)((sp.np + kBlock - 1) / kBlock)), block(kBlock);
  if (through)
    hipLaunchKernelGGL((k_backward<T, CELL, true>), grid, block, 0, st, A);
  else
    hipLaunchKernelGGL((k_backward<T, CELL, false>), grid, block, 0, st, A);
  return hipGetLastError();
}

}  // namespace

size_t backward_table_offset(int64_t np) { return 256 + (((size_t)4 * (size_t)np + 255) / 256) * 256; }

size_t backward_workspace_bytes(const Grid& g, int64_t np, bool f32) {
  return backward_table_offset(np) + (size_t)g.nn * kGS * (f32 ? sizeof(float) : sizeof(double));
}

hipError_t launch_backward(const Grid& g, bool f32, const SpeciesArgs& sp, const void* E, const void* B,
                           const void* gJ, const void* gM, void* const gpos[3], void* const gvel[3], void* gE,
                           void* gB, bool through_mover, bool offset_grad, void* ws, hipStream_t st) {
  if (sp.np == 0) return hipSuccess;
  if (f32) return launch_T<float, true>(g, sp, E, B, gJ, gM, gpos, gvel, gE, gB, through_mover, offset_grad, ws, st);
  return launch_T<double, false>(g, sp, E, B, gJ, gM, gpos, gvel, gE, gB, through_mover, false, ws, st);
}

}  // namespace ecsim
