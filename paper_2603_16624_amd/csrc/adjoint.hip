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
#include "internal.h"

namespace ecsim {

namespace {

constexpr int kBlock = 256;

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

template <typename T, bool CELL, bool THROUGH>
__global__ void __launch_bounds__(kBlock) k_backward(
    Grid g, int np, const T* __restrict__ p0, const T* __restrict__ p1, const T* __restrict__ p2,
    const int32_t* __restrict__ cell, const T* __restrict__ v0, const T* __restrict__ v1, const T* __restrict__ v2,
    const T* __restrict__ q, T q_const, T beta, T dth0, T dth1, T dth2, const T* __restrict__ E,
    const T* __restrict__ B, const T* __restrict__ gJ, const T* __restrict__ gM, T* __restrict__ gx0,
    T* __restrict__ gx1, T* __restrict__ gx2, T* __restrict__ gv0, T* __restrict__ gv1, T* __restrict__ gv2,
    T* __restrict__ gE, T* __restrict__ gB, bool offset_grad) {
  // every lane runs (the gradient scatter works across the wavefront); lanes
  // past the end recompute the last particle and store nothing
  const int lane = threadIdx.x & 63;
  const bool valid = blockIdx.x * kBlock + threadIdx.x < np;
  const int p = valid ? blockIdx.x * kBlock + threadIdx.x : np - 1;
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
  for (int ca = 0; ca < 8; ++ca) {
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

template <typename T, bool CELL>
hipError_t launch_T(const Grid& g, const SpeciesArgs& sp, const void* E, const void* B, const void* gJ,
                    const void* gM, void* const gpos[3], void* const gvel[3], void* gE, void* gB, bool through,
                    bool offset_grad, hipStream_t st) {
  const double beta = sp.qom * g.dt / 2.0;
  dim3 grid((unsigned)((sp.np + kBlock - 1) / kBlock)), block(kBlock);
  auto args = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, block, 0, st, g, sp.np, (const T*)sp.pos[0], (const T*)sp.pos[1],
                       (const T*)sp.pos[2], (const int32_t*)sp.cell, (const T*)sp.vel[0], (const T*)sp.vel[1],
                       (const T*)sp.vel[2], (const T*)sp.q, (T)sp.q_const, (T)beta, (T)(g.pdt[0] / g.hx),
                       (T)(g.pdt[1] / g.hy), (T)(g.pdt[2] / g.hz), (const T*)E, (const T*)B, (const T*)gJ, (const T*)gM,
                       (T*)gpos[0], (T*)gpos[1], (T*)gpos[2], (T*)gvel[0], (T*)gvel[1], (T*)gvel[2], (T*)gE,
                       (T*)gB, offset_grad);
  };
  if (through)
    args(k_backward<T, CELL, true>);
  else
    args(k_backward<T, CELL, false>);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_backward(const Grid& g, bool f32, const SpeciesArgs& sp, const void* E, const void* B,
                           const void* gJ, const void* gM, void* const gpos[3], void* const gvel[3], void* gE,
                           void* gB, bool through_mover, bool offset_grad, hipStream_t st) {
  if (sp.np == 0) return hipSuccess;
  if (f32) return launch_T<float, true>(g, sp, E, B, gJ, gM, gpos, gvel, gE, gB, through_mover, offset_grad, st);
  return launch_T<double, false>(g, sp, E, B, gJ, gM, gpos, gvel, gE, gB, through_mover, false, st);
}

}  // namespace ecsim
