// Device-side building blocks of the ECsim hot path (gfx950).
//
// One inline routine computes each quantity -- interpolation stencil, field
// gather, rotation matrix -- so that the mover, the moment deposit and the
// adjoint share them (the scheme conserves energy only if the mover and the
// moments use the same alpha_p and W_pN). In FP64 the mover and the deposit
// obtain bit-identical alpha_p. In FP32 they agree to rounding only: the mover
// evaluates the velocity update in FP64 and rounds v^{n+1} once (see
// advance_velocity), while the deposit forms alpha_p in FP32 with the charge
// factors folded into 1/(1 + |beta B|^2). Both differences are unbiased
// roundings of the same exact alpha_p, so the energy error they add is a
// random walk of FP32 rounding size per particle, not a drift.
// The library is compiled with -ffp-contract=off; fused multiply-adds appear
// only where written explicitly.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace ecsim {

// Exact division by a runtime constant d >= 1 for numerators below 2^31
// (every cell index): with L = ceil(log2 d) and m = ceil(2^(31+L) / d), which
// lies in [2^31, 2^32), n / d is the high word of n m shifted right by L - 1.
// The rounding error of m adds less than n / 2^(31+L) < 1/d to n / d, too
// little to cross an integer. d = 1 passes n through. Branch-free: one
// multiply-high and a shift in place of the division sequence.
struct FastDiv {
  uint32_t d, m;
  int s;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f{d, 0u, 0};
  if (d > 1) {
    int L = 0;
    while ((1ull << L) < d) ++L;
    f.m = (uint32_t)(((1ull << (31 + L)) + d - 1) / d);
    f.s = L - 1;
  }
  return f;
}

__device__ __forceinline__ uint32_t fast_div(uint32_t n, FastDiv f) {
  return f.d == 1 ? n : (__umulhi(n, f.m) >> f.s);
}

__device__ __forceinline__ uint32_t fast_divmod(uint32_t n, FastDiv f, uint32_t& r) {
  const uint32_t q = fast_div(n, f);
  r = n - q * f.d;
  return q;
}

struct Grid {
  int nx, ny, nz;
  double hx, hy, hz, dt;
  int64_t nn;        // nodes = cells
  double V;          // control volume of a node
  FastDiv div_x;     // by nx
  FastDiv div_xy;    // by nx * ny
  double pdt[3];     // position push time step per dimension: dt, or 0 along a
                     // dimension of one cell (reduced runs keep positions there)
  int* nonfinite;    // the device's non-finite flag (set, never cleared, by kernels)
};

// true unless x is a NaN or an infinity
template <typename T>
__device__ __forceinline__ bool finite(T x) {
  return __builtin_isfinite(x);
}

// Records that a kernel produced a non-finite value (a vector atomic on the
// flag; lanes without one do nothing).
__device__ __forceinline__ void note_nonfinite(const Grid& g, bool bad) {
  if (bad && g.nonfinite) atomicOr(g.nonfinite, 1);
}

template <typename T> struct Vec3 { T x, y, z; };

// Interpolation stencil of one particle: lower node (N^-) per dimension and
// the linear weights w[d][0] (N^-) and w[d][1] (N^+ = N^- + 1); the eight
// weights of the 2x2x2 stencil are products of one factor per dimension.
template <typename T>
struct Stencil {
  int i[3];          // lower node, in [0, n)
  int ip[3];         // upper node, wrapped
  T w0[3], w1[3];    // 1 - xi, xi
};

__device__ __forceinline__ int wrap_up(int i, int n) { return (i + 1 == n) ? 0 : i + 1; }

// i in [-n, 2n) taken periodically into [0, n)
__device__ __forceinline__ int wrap_once(int i, int n) {
  i += i < 0 ? n : 0;
  return i >= n ? i - n : i;
}

// FP64 form: absolute position in [0, L).
__device__ __forceinline__ Stencil<double> stencil_abs(const Grid& g, double x, double y, double z) {
  Stencil<double> s;
  const double u[3] = {x / g.hx, y / g.hy, z / g.hz};
  const int n[3] = {g.nx, g.ny, g.nz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double fl = floor(u[d]);
    double xi = u[d] - fl;
    int i = (int)fl;
    if (i >= n[d] || i < 0) {   // positions are expected in [0, L); wrap anything else
      i %= n[d];
      if (i < 0) i += n[d];
    }
    s.i[d] = i;
    s.ip[d] = wrap_up(i, n[d]);
    s.w0[d] = 1.0 - xi;
    s.w1[d] = xi;
  }
  return s;
}

// FP32 form: int32 cell index + in-cell offsets in [0, 1).
__device__ __forceinline__ void decode_cell(const Grid& g, int cell, int& ix, int& iy, int& iz) {
  uint32_t r, r2;
  iz = (int)fast_divmod((uint32_t)cell, g.div_xy, r);
  iy = (int)fast_divmod(r, g.div_x, r2);
  ix = (int)r2;
}

__device__ __forceinline__ Stencil<float> stencil_cell(const Grid& g, int cell, float ox, float oy, float oz) {
  Stencil<float> s;
  int ix, iy, iz;
  decode_cell(g, cell, ix, iy, iz);
  s.i[0] = ix; s.i[1] = iy; s.i[2] = iz;
  s.ip[0] = wrap_up(ix, g.nx); s.ip[1] = wrap_up(iy, g.ny); s.ip[2] = wrap_up(iz, g.nz);
  s.w1[0] = ox; s.w1[1] = oy; s.w1[2] = oz;
  s.w0[0] = 1.0f - ox; s.w0[1] = 1.0f - oy; s.w0[2] = 1.0f - oz;
  return s;
}

// node of corner a = ax + 2 ay + 4 az
template <typename T>
__device__ __forceinline__ int64_t corner_node(const Grid& g, const Stencil<T>& s, int a) {
  int ix = (a & 1) ? s.ip[0] : s.i[0];
  int iy = (a & 2) ? s.ip[1] : s.i[1];
  int iz = (a & 4) ? s.ip[2] : s.i[2];
  return ix + (int64_t)g.nx * (iy + (int64_t)g.ny * iz);
}

template <typename T>
__device__ __forceinline__ T corner_weight(const Stencil<T>& s, int a) {
  T wx = (a & 1) ? s.w1[0] : s.w0[0];
  T wy = (a & 2) ? s.w1[1] : s.w0[1];
  T wz = (a & 4) ? s.w1[2] : s.w0[2];
  return (wx * wy) * wz;
}

// All eight weights and nodes.
template <typename T>
__device__ __forceinline__ void corners(const Grid& g, const Stencil<T>& s, T W[8], int64_t node[8]) {
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    W[a] = corner_weight(s, a);
    node[a] = corner_node(g, s, a);
  }
}

// F_p = sum_a W_a F[node(a)] for a [3][Nn] field.
template <typename T>
__device__ __forceinline__ Vec3<T> gather(const T* __restrict__ F, int64_t nn, const T W[8], const int64_t node[8]) {
  Vec3<T> r{T(0), T(0), T(0)};
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    r.x = fma(W[a], F[node[a]], r.x);
    r.y = fma(W[a], F[nn + node[a]], r.y);
    r.z = fma(W[a], F[2 * nn + node[a]], r.z);
  }
  return r;
}

// Rotation matrix of Eq. 2 for the Lorentz force q (E + v x B), c = 1:
//   alpha = (I - beta [B x] + beta^2 B B^T) / (1 + beta^2 |B|^2),
// [B x] u = B x u; alpha u solves vbar - beta vbar x B = u. Row major a[3i+j].
template <typename T>
__device__ __forceinline__ void rotation(Vec3<T> B, T beta, T a[9]) {
  T bx = beta * B.x, by = beta * B.y, bz = beta * B.z;
  T den = T(1) + ((bx * bx + by * by) + bz * bz);
  // FP32: the hardware reciprocal (1 ulp) in place of the correctly rounded
  // division sequence; FP64 divides
  T inv;
  if constexpr (sizeof(T) == 4) inv = __builtin_amdgcn_rcpf(den);
  else inv = T(1) / den;
  a[0] = (T(1) + bx * bx) * inv;
  a[1] = (bx * by + bz) * inv;
  a[2] = (bx * bz - by) * inv;
  a[3] = (by * bx - bz) * inv;
  a[4] = (T(1) + by * by) * inv;
  a[5] = (by * bz + bx) * inv;
  a[6] = (bz * bx + by) * inv;
  a[7] = (bz * by - bx) * inv;
  a[8] = (T(1) + bz * bz) * inv;
}

template <typename T>
__device__ __forceinline__ Vec3<T> matvec(const T a[9], Vec3<T> u) {
  return Vec3<T>{(a[0] * u.x + a[1] * u.y) + a[2] * u.z,
                 (a[3] * u.x + a[4] * u.y) + a[5] * u.z,
                 (a[6] * u.x + a[7] * u.y) + a[8] * u.z};
}

// Velocity update of Eqs. 4-5: u = v + beta E_p, vbar = alpha u,
// v^{n+1} = 2 vbar - v.
template <typename T>
__device__ __forceinline__ Vec3<T> velocity_update(const T a[9], Vec3<T> v, Vec3<T> Ep, T beta, Vec3<T>& u) {
  u = Vec3<T>{v.x + beta * Ep.x, v.y + beta * Ep.y, v.z + beta * Ep.z};
  Vec3<T> vb = matvec(a, u);
  return Vec3<T>{T(2) * vb.x - v.x, T(2) * vb.y - v.y, T(2) * vb.z - v.z};
}

// The mover's step of Eqs. 3-5 from the gathered fields. In the FP32 form
// the update is evaluated in FP64 and v^{n+1} is rounded once: the map
// v -> (2 alpha - I) v is a rotation, but with alpha rounded to FP32 it
// scales |v| by 1 + O(1e-7), and where B is nearly uniform all particles share
// that rounding, so the kinetic energy would drift one way every step. A single
// rounding of the result is unbiased and averages out over the particles.
// The FP64 evaluation writes alpha u out directly, with b = beta B:
//   vbar = (u + u x b + b (b . u)) / (1 + |b|^2),  u = v + beta E_p,
// and 1/(1 + |b|^2) from the hardware reciprocal refined by two Newton steps
// (each squares the relative error, from 2^-26 to below the FP64 rounding).
// Every FP32 mover (grouped, stray, any order) and the adjoint's recompute of
// the push call this routine, so they move a particle identically.
template <typename T>
__device__ __forceinline__ Vec3<T> advance_velocity(Vec3<T> Bp, T beta, Vec3<T> v, Vec3<T> Ep) {
  if constexpr (sizeof(T) == 4) {
    const double bt = beta;
    const double bx = bt * (double)Bp.x, by = bt * (double)Bp.y, bz = bt * (double)Bp.z;
    const double den = fma(bx, bx, fma(by, by, fma(bz, bz, 1.0)));
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    r = fma(r, fma(-den, r, 1.0), r);
    const double vx = v.x, vy = v.y, vz = v.z;
    const double ux = fma(bt, (double)Ep.x, vx), uy = fma(bt, (double)Ep.y, vy), uz = fma(bt, (double)Ep.z, vz);
    const double bu = fma(bx, ux, fma(by, uy, bz * uz));
    const double wx = fma(bx, bu, ux + fma(uy, bz, -uz * by));
    const double wy = fma(by, bu, uy + fma(uz, bx, -ux * bz));
    const double wz = fma(bz, bu, uz + fma(ux, by, -uy * bx));
    return Vec3<T>{(T)fma(2.0 * r, wx, -vx), (T)fma(2.0 * r, wy, -vy), (T)fma(2.0 * r, wz, -vz)};
  } else {
    T a[9];
    rotation(Bp, beta, a);
    Vec3<T> u;
    return velocity_update(a, v, Ep, beta, u);
  }
}

// Position push of Eq. 8, FP64 form: x + dt v wrapped into [0, L); a result
// that rounds to L is stored as 0.
__device__ __forceinline__ double push_abs(double x, double dt, double v, double L) {
  double y = x + dt * v;
  double k = floor(y / L);
  double r = y - k * L;
  if (r >= L) r -= L;
  if (r < 0.0) r += L;
  if (r >= L) r = 0.0;
  return r;
}

// Position push of Eq. 8, FP32 form along one dimension: offset + dt v / h,
// carrying whole cells into the (periodic) cell index.
__device__ __forceinline__ float push_offset(float o, float v, float dth, int& idx, int n) {
  float u = o + v * dth;
  float fl = floorf(u);
  float r = u - fl;
  int shift = (int)fl;
  if (r >= 1.0f) { r = 0.0f; shift += 1; }
  int j = idx + shift;
  j += j < 0 ? n : 0;        // one period either way without a division
  j -= j >= n ? n : 0;
  if (j < 0 || j >= n) {     // more than one period in a step
    j %= n;
    if (j < 0) j += n;
  }
  idx = j;
  return r;
}

// d(weight of corner a)/d(xi_d)
template <typename T>
__device__ __forceinline__ void weight_grad(const Stencil<T>& s, const T gW[8], T gxi[3]) {
  gxi[0] = gxi[1] = gxi[2] = T(0);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    T wx = (a & 1) ? s.w1[0] : s.w0[0];
    T wy = (a & 2) ? s.w1[1] : s.w0[1];
    T wz = (a & 4) ? s.w1[2] : s.w0[2];
    T sx = (a & 1) ? T(1) : T(-1);
    T sy = (a & 2) ? T(1) : T(-1);
    T sz = (a & 4) ? T(1) : T(-1);
    gxi[0] += gW[a] * (sx * (wy * wz));
    gxi[1] += gW[a] * (sy * (wx * wz));
    gxi[2] += gW[a] * (sz * (wx * wy));
  }
}

// Vector-Jacobian product of the rotation matrix of Eq. 2 with respect to B:
// given G = dL/d alpha (row major), returns dL/dB. With b = beta B,
// D = 1 + |b|^2 and N = I + b b^T - [b x]:
//   dL/db_k = ((G b)_k + (G^T b)_k + eps_kij G_ij - 2 b_k <G, alpha>) / D.
template <typename T>
__device__ __forceinline__ Vec3<T> rotation_vjp(const T a[9], Vec3<T> B, T beta, const T G[9]) {
  T bx = beta * B.x, by = beta * B.y, bz = beta * B.z;
  T den = T(1) + ((bx * bx + by * by) + bz * bz);
  T ga = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) ga += G[i] * a[i];
  T gbx = (G[0] * bx + G[1] * by + G[2] * bz) + (G[0] * bx + G[3] * by + G[6] * bz) + (G[5] - G[7]);
  T gby = (G[3] * bx + G[4] * by + G[5] * bz) + (G[1] * bx + G[4] * by + G[7] * bz) + (G[6] - G[2]);
  T gbz = (G[6] * bx + G[7] * by + G[8] * bz) + (G[2] * bx + G[5] * by + G[8] * bz) + (G[1] - G[3]);
  T two_ga = T(2) * ga;
  // FP32: the hardware reciprocal (1 ulp); FP64 divides
  T inv;
  if constexpr (sizeof(T) == 4) inv = __builtin_amdgcn_rcpf(den);
  else inv = T(1) / den;
  return Vec3<T>{beta * ((gbx - two_ga * bx) * inv), beta * ((gby - two_ga * by) * inv),
                 beta * ((gbz - two_ga * bz) * inv)};
}

// The 14 stored neighbour offsets (see the header): o_k for k = 0..13.
__host__ __device__ __forceinline__ void offset14(int k, int& ox, int& oy, int& oz) {
  if (k == 0) { ox = 0; oy = 0; oz = 0; }
  else if (k == 1) { ox = 1; oy = 0; oz = 0; }
  else if (k < 5) { ox = k - 3; oy = 1; oz = 0; }
  else { int r = k - 5; ox = r % 3 - 1; oy = r / 3 - 1; oz = 1; }
}

// Stored block of the ordered corner pair (a, b) of one cell: returns k and
// whether the block sits at node(a) (true) or node(b) (false). Offsets between
// corners are b - a in {-1,0,1}^3; exactly one of o and -o is stored (o != 0).
__device__ __forceinline__ int pair_block(int a, int b, bool& at_a) {
  int ox = (b & 1) - (a & 1), oy = ((b >> 1) & 1) - ((a >> 1) & 1), oz = ((b >> 2) & 1) - ((a >> 2) & 1);
  bool stored = (oz > 0) || (oz == 0 && (oy > 0 || (oy == 0 && ox >= 0)));
  at_a = stored;
  if (!stored) { ox = -ox; oy = -oy; oz = -oz; }
  if (oz == 0 && oy == 0) return ox == 0 ? 0 : 1;
  if (oz == 0) return 3 + ox;
  return 5 + (ox + 1) + 3 * (oy + 1);
}

// Brick origin of workgroup blockIdx.x; blocks are spread so that each XCD
// gets contiguous bricks.
template <int TX, int TY, int TZ>
__device__ __forceinline__ void brick_origin(int ntx, int nty, int ntz, int& x0, int& y0, int& z0) {
  const int ntiles = ntx * nty * ntz;
  int b = blockIdx.x;
  constexpr int nxcd = 8;
  const int per = ntiles / nxcd;
  if (per * nxcd == ntiles) b = (b % nxcd) * per + b / nxcd;
  x0 = (b % ntx) * TX;
  y0 = ((b / ntx) % nty) * TY;
  z0 = (b / (ntx * nty)) * TZ;
}

}  // namespace ecsim
