// Node-grid kernels: matrix-free mass-matrix apply (Eq. 7), staggered curls,
// centre-to-node averaging, and the FP64 vector kernels of the GMRES solve.
#include <algorithm>
#include "internal.h"

namespace ecsim {

namespace {

constexpr int kBlock = 256;
inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ int wp(int i, int n) { return i + 1 == n ? 0 : i + 1; }   // i + 1 mod n
__device__ __forceinline__ int wm(int i, int n) { return i == 0 ? n - 1 : i - 1; }   // i - 1 mod n
__device__ __forceinline__ int shift(int i, int o, int n) { return o > 0 ? wp(i, n) : (o < 0 ? wm(i, n) : i); }

// ---------------------------------------------------------------------------
// y = a (M x) + b y with the 14 stored blocks (block k at g couples g and
// g + o_k; the same block, untransposed, couples g + o_k back to g).
// One thread per node; the [14][9][Nn] layout makes every M read coalesced.
// Workgroups go to the 8 XCDs in turn; each XCD is given a contiguous eighth
// of the nodes, so that the blocks read again at g - o (up to one z-plane
// back) are still in that XCD's L2.
// ---------------------------------------------------------------------------
template <typename TM>
__global__ void __launch_bounds__(kBlock) k_mass_apply(Grid g, const TM* __restrict__ M, const double* __restrict__ x,
                                                       double a, double b, double* __restrict__ y) {
  const int64_t nn = g.nn;
  int blk = blockIdx.x;
  if ((gridDim.x & 7) == 0) blk = (blk & 7) * (gridDim.x >> 3) + (blk >> 3);
  const int64_t gid = blk * (int64_t)kBlock + threadIdx.x;
  if (gid >= nn) return;
  int ix, iy, iz;
  decode_cell(g, (int)gid, ix, iy, iz);
  double y0 = 0.0, y1 = 0.0, y2 = 0.0;
#pragma unroll
  for (int k = 0; k < 14; ++k) {
    int ox, oy, oz;
    offset14(k, ox, oy, oz);
    const TM* Mk = M + (int64_t)k * 9 * nn;
    {
      int64_t gp = shift(ix, ox, g.nx) + (int64_t)g.nx * (shift(iy, oy, g.ny) + (int64_t)g.ny * shift(iz, oz, g.nz));
      double e0 = x[gp], e1 = x[nn + gp], e2 = x[2 * nn + gp];
      y0 = fma((double)Mk[0 * nn + gid], e0, y0);
      y0 = fma((double)Mk[1 * nn + gid], e1, y0);
      y0 = fma((double)Mk[2 * nn + gid], e2, y0);
      y1 = fma((double)Mk[3 * nn + gid], e0, y1);
      y1 = fma((double)Mk[4 * nn + gid], e1, y1);
      y1 = fma((double)Mk[5 * nn + gid], e2, y1);
      y2 = fma((double)Mk[6 * nn + gid], e0, y2);
      y2 = fma((double)Mk[7 * nn + gid], e1, y2);
      y2 = fma((double)Mk[8 * nn + gid], e2, y2);
    }
    if (k > 0) {
      int64_t gm = shift(ix, -ox, g.nx) + (int64_t)g.nx * (shift(iy, -oy, g.ny) + (int64_t)g.ny * shift(iz, -oz, g.nz));
      double e0 = x[gm], e1 = x[nn + gm], e2 = x[2 * nn + gm];
      y0 = fma((double)Mk[0 * nn + gm], e0, y0);
      y0 = fma((double)Mk[1 * nn + gm], e1, y0);
      y0 = fma((double)Mk[2 * nn + gm], e2, y0);
      y1 = fma((double)Mk[3 * nn + gm], e0, y1);
      y1 = fma((double)Mk[4 * nn + gm], e1, y1);
      y1 = fma((double)Mk[5 * nn + gm], e2, y1);
      y2 = fma((double)Mk[6 * nn + gm], e0, y2);
      y2 = fma((double)Mk[7 * nn + gm], e1, y2);
      y2 = fma((double)Mk[8 * nn + gm], e2, y2);
    }
  }
  if (b == 0.0) {
    y[gid] = a * y0;
    y[nn + gid] = a * y1;
    y[2 * nn + gid] = a * y2;
  } else {
    y[gid] = a * y0 + b * y[gid];
    y[nn + gid] = a * y1 + b * y[nn + gid];
    y[2 * nn + gid] = a * y2 + b * y[2 * nn + gid];
  }
}

// ---------------------------------------------------------------------------
// staggered curls: E on nodes, B on cell centres; each derivative averages the
// four edge differences parallel to its axis (curl_N = curl_C^T).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_curl_C(Grid g, const double* __restrict__ E, double* __restrict__ out) {
  const int64_t nn = g.nn;
  const int64_t c = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (c >= nn) return;
  int cx, cy, cz;
  decode_cell(g, (int)c, cx, cy, cz);
  const int xs[2] = {cx, wp(cx, g.nx)}, ys[2] = {cy, wp(cy, g.ny)}, zs[2] = {cz, wp(cz, g.nz)};
  double d[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // d[axis][component]
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      int64_t x1 = xs[1] + (int64_t)g.nx * (ys[a] + (int64_t)g.ny * zs[b]);
      int64_t x0 = xs[0] + (int64_t)g.nx * (ys[a] + (int64_t)g.ny * zs[b]);
      int64_t y1 = xs[a] + (int64_t)g.nx * (ys[1] + (int64_t)g.ny * zs[b]);
      int64_t y0 = xs[a] + (int64_t)g.nx * (ys[0] + (int64_t)g.ny * zs[b]);
      int64_t z1 = xs[a] + (int64_t)g.nx * (ys[b] + (int64_t)g.ny * zs[1]);
      int64_t z0 = xs[a] + (int64_t)g.nx * (ys[b] + (int64_t)g.ny * zs[0]);
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        const double* F = E + comp * nn;
        d[0][comp] += F[x1] - F[x0];
        d[1][comp] += F[y1] - F[y0];
        d[2][comp] += F[z1] - F[z0];
      }
    }
  const double ix = 1.0 / (4.0 * g.hx), iy = 1.0 / (4.0 * g.hy), iz = 1.0 / (4.0 * g.hz);
  out[c] = d[1][2] * iy - d[2][1] * iz;
  out[nn + c] = d[2][0] * iz - d[0][2] * ix;
  out[2 * nn + c] = d[0][1] * ix - d[1][0] * iy;
}

__device__ __forceinline__ void curl_N_at(const Grid& g, const double* __restrict__ B, int64_t nd, double r[3]) {
  const int64_t nn = g.nn;
  int gx, gy, gz;
  decode_cell(g, (int)nd, gx, gy, gz);
  // cells around node g: g - 1 + a
  const int xs[2] = {wm(gx, g.nx), gx}, ys[2] = {wm(gy, g.ny), gy}, zs[2] = {wm(gz, g.nz), gz};
  double d[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      int64_t x1 = xs[1] + (int64_t)g.nx * (ys[a] + (int64_t)g.ny * zs[b]);
      int64_t x0 = xs[0] + (int64_t)g.nx * (ys[a] + (int64_t)g.ny * zs[b]);
      int64_t y1 = xs[a] + (int64_t)g.nx * (ys[1] + (int64_t)g.ny * zs[b]);
      int64_t y0 = xs[a] + (int64_t)g.nx * (ys[0] + (int64_t)g.ny * zs[b]);
      int64_t z1 = xs[a] + (int64_t)g.nx * (ys[b] + (int64_t)g.ny * zs[1]);
      int64_t z0 = xs[a] + (int64_t)g.nx * (ys[b] + (int64_t)g.ny * zs[0]);
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        const double* F = B + comp * nn;
        d[0][comp] += F[x1] - F[x0];
        d[1][comp] += F[y1] - F[y0];
        d[2][comp] += F[z1] - F[z0];
      }
    }
  const double ix = 1.0 / (4.0 * g.hx), iy = 1.0 / (4.0 * g.hy), iz = 1.0 / (4.0 * g.hz);
  r[0] = d[1][2] * iy - d[2][1] * iz;
  r[1] = d[2][0] * iz - d[0][2] * ix;
  r[2] = d[0][1] * ix - d[1][0] * iy;
}

// out = E + ctd2 * curl_N(cC), cC = curl_C E (the curl-curl part of A E)
__global__ void __launch_bounds__(kBlock) k_field_op_curl(Grid g, const double* __restrict__ E,
                                                          const double* __restrict__ cC, double ctd2,
                                                          double* __restrict__ out) {
  const int64_t nd = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (nd >= g.nn) return;
  double r[3];
  curl_N_at(g, cC, nd, r);
  for (int c = 0; c < 3; ++c) out[c * g.nn + nd] = E[c * g.nn + nd] + ctd2 * r[c];
}

// b = E_n + c_j J + c_b curl_N(BC)
template <typename TJ>
__global__ void __launch_bounds__(kBlock) k_rhs(Grid g, const double* __restrict__ En, const TJ* __restrict__ J,
                                                const double* __restrict__ BC, double c_j, double c_b,
                                                double* __restrict__ b) {
  const int64_t nd = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (nd >= g.nn) return;
  double r[3];
  curl_N_at(g, BC, nd, r);
  for (int c = 0; c < 3; ++c) b[c * g.nn + nd] = (En[c * g.nn + nd] + c_j * (double)J[c * g.nn + nd]) + c_b * r[c];
}

// E^{n+1} = 2 E^{n+theta} - E^n; B^{n+1} = 2 (B^n - ctd curl_C E^{n+theta}) - B^n
__global__ void __launch_bounds__(kBlock) k_finish(int64_t n3, const double* __restrict__ En,
                                                   const double* __restrict__ Et, const double* __restrict__ BCn,
                                                   const double* __restrict__ cc, double ctd,
                                                   double* __restrict__ En1, double* __restrict__ BCn1) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n3) return;
  En1[i] = 2.0 * Et[i] - En[i];
  double bt = BCn[i] - ctd * cc[i];
  BCn1[i] = 2.0 * bt - BCn[i];
}

__global__ void __launch_bounds__(kBlock) k_centres_to_nodes(Grid g, const double* __restrict__ BC,
                                                             double* __restrict__ BN, float* __restrict__ BN32) {
  const int64_t nd = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (nd >= g.nn) return;
  int gx, gy, gz;
  decode_cell(g, (int)nd, gx, gy, gz);
  const int xs[2] = {wm(gx, g.nx), gx}, ys[2] = {wm(gy, g.ny), gy}, zs[2] = {wm(gz, g.nz), gz};
  for (int comp = 0; comp < 3; ++comp) {
    double s = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c) s += BC[comp * g.nn + xs[a] + (int64_t)g.nx * (ys[b] + (int64_t)g.ny * zs[c])];
    double v = s / 8.0;
    if (BN) BN[comp * g.nn + nd] = v;
    if (BN32) BN32[comp * g.nn + nd] = (float)v;
  }
}

__global__ void __launch_bounds__(kBlock) k_to_f32(int64_t n, const double* __restrict__ s, float* __restrict__ d) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) d[i] = (float)s[i];
}

// ---------------------------------------------------------------------------
// FP64 vector kernels (deterministic: fixed grid, tree reductions)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_reduce(double v) {
  __shared__ double red[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

// partial[v * kDotBlocks + blk] = sum over this block's slice of V_v . w
__global__ void __launch_bounds__(kBlock) k_dots_partial(const double* __restrict__ V, int64_t ld, int nv,
                                                         const double* __restrict__ w, int64_t n,
                                                         double* __restrict__ partial) {
  for (int v = 0; v < nv; ++v) {
    const double* Vv = V + v * ld;
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
      s = fma(Vv[i], w[i], s);
    s = block_reduce(s);
    if (threadIdx.x == 0) partial[v * kDotBlocks + blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(kBlock) k_dots_final(const double* __restrict__ partial, int nv,
                                                       double* __restrict__ out) {
  // one block per vector
  const int v = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < kDotBlocks; i += kBlock) s += partial[v * kDotBlocks + i];
  s = block_reduce(s);
  if (threadIdx.x == 0) out[v] = s;
}

__global__ void __launch_bounds__(kBlock) k_sumsq_partial(const double* __restrict__ x, int64_t n,
                                                          double* __restrict__ partial) {
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    s = fma(x[i], x[i], s);
  s = block_reduce(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) k_sumsq_final(const double* __restrict__ partial, double scale,
                                                        double* __restrict__ out, int accumulate) {
  double s = 0.0;
  for (int i = threadIdx.x; i < kDotBlocks; i += kBlock) s += partial[i];
  s = block_reduce(s);
  if (threadIdx.x == 0) *out = accumulate ? *out + scale * s : scale * s;
}

struct Coefs {
  double c[kMaxRestart + 1];
};

__global__ void __launch_bounds__(kBlock) k_sub_combo(const double* __restrict__ V, int64_t ld, int nv, Coefs coef,
                                                      double* __restrict__ w, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n) return;
  double s = w[i];
  for (int v = 0; v < nv; ++v) s -= coef.c[v] * V[v * ld + i];
  w[i] = s;
}

// w -= sum_v coef[v] V_v with the coefficients in device memory
__global__ void __launch_bounds__(kBlock) k_sub_combo_dev(const double* __restrict__ V, int64_t ld, int nv,
                                                          const double* __restrict__ coef, double* __restrict__ w,
                                                          int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n) return;
  double s = w[i];
  for (int v = 0; v < nv; ++v) s -= coef[v] * V[v * ld + i];
  w[i] = s;
}

// out = w / sqrt(*nrm2) (zeros when the norm is zero: a Krylov breakdown)
__global__ void __launch_bounds__(kBlock) k_normalize(const double* __restrict__ w, const double* __restrict__ nrm2,
                                                      double* __restrict__ out, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n) return;
  const double s = *nrm2;
  out[i] = s > 0.0 ? w[i] / sqrt(s) : 0.0;
}

// One Arnoldi column on the device (one thread): H[:, j] from the two
// Gram-Schmidt passes and the new vector's norm, the earlier Givens rotations
// applied to it, a new rotation that zeroes H[j+1][j], and the rotated
// right-hand side g. hist[j] = |g[j+1]|, the residual norm of the least-squares
// problem after j + 1 steps. Once that norm is below thresh (or the Krylov
// space broke down), state[0] = 0 and later calls leave everything as is, so
// steps launched past convergence change nothing. state[1] = columns used.
__global__ void k_givens(int j, int m, double* __restrict__ H, double* __restrict__ cs, double* __restrict__ sn,
                         double* __restrict__ gv, const double* __restrict__ h1, const double* __restrict__ h2,
                         const double* __restrict__ hn2, double thresh, int* __restrict__ state,
                         double* __restrict__ hist) {
  if (state[0] == 0) {
    hist[j] = -1.0;
    return;
  }
  const double hn = sqrt(*hn2 > 0.0 ? *hn2 : 0.0);
  for (int i = 0; i <= j; ++i) H[(int64_t)i * m + j] = h1[i] + h2[i];
  H[(int64_t)(j + 1) * m + j] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = H[(int64_t)i * m + j], b = H[(int64_t)(i + 1) * m + j];
    H[(int64_t)i * m + j] = cs[i] * a + sn[i] * b;
    H[(int64_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
  }
  const double a = H[(int64_t)j * m + j], b = H[(int64_t)(j + 1) * m + j];
  const double rr = hypot(a, b);
  cs[j] = rr > 0.0 ? a / rr : 1.0;
  sn[j] = rr > 0.0 ? b / rr : 0.0;
  H[(int64_t)j * m + j] = rr;
  H[(int64_t)(j + 1) * m + j] = 0.0;
  gv[j + 1] = -sn[j] * gv[j];
  gv[j] = cs[j] * gv[j];
  hist[j] = fabs(gv[j + 1]);
  state[1] = j + 1;
  if (hist[j] <= thresh || hn == 0.0) state[0] = 0;
}

// start of a restart cycle: g = (beta, 0, ...), one active iteration state
__global__ void k_gmres_start(int m, double beta, double* __restrict__ gv, int* __restrict__ state) {
  for (int i = 0; i <= m; ++i) gv[i] = i == 0 ? beta : 0.0;
  state[0] = 1;
  state[1] = 0;
}

// back substitution of the j x j triangle H y = g (one thread); writes -y
__global__ void k_backsolve(const double* __restrict__ H, const double* __restrict__ gv, int m, int j,
                            double* __restrict__ ny) {
  for (int i = j - 1; i >= 0; --i) {
    double s = gv[i];
    for (int k = i + 1; k < j; ++k) s += H[(int64_t)i * m + k] * ny[k];   // ny[k] = -y[k]
    ny[i] = -(s / H[(int64_t)i * m + i]);
  }
}

__global__ void __launch_bounds__(kBlock) k_axpby(int64_t n, double a, const double* __restrict__ x, double b,
                                                  double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

__global__ void __launch_bounds__(kBlock) k_scale_copy(int64_t n, double a, const double* __restrict__ x,
                                                       double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// the non-finite flag, read and cleared in stream order
__global__ void k_take_flag(int* __restrict__ flag, int32_t* __restrict__ out) {
  out[0] = flag[0];
  flag[0] = 0;
}

__global__ void __launch_bounds__(kBlock) k_zero(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// 16-byte stores over a fixed grid, for large 16-byte aligned fills
__global__ void __launch_bounds__(kBlock) k_zero16(uint4* __restrict__ p, int64_t n16) {
  const uint4 z = {0u, 0u, 0u, 0u};
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n16; i += (int64_t)gridDim.x * kBlock) p[i] = z;
}

}  // namespace

hipError_t launch_mass_apply(const Grid& g, bool f32, const void* M, const double* x, double a, double b, double* y,
                             hipStream_t st) {
  if (f32)
    hipLaunchKernelGGL(k_mass_apply<float>, dim3(nblocks(g.nn, kBlock)), dim3(kBlock), 0, st, g, (const float*)M, x,
                       a, b, y);
  else
    hipLaunchKernelGGL(k_mass_apply<double>, dim3(nblocks(g.nn, kBlock)), dim3(kBlock), 0, st, g, (const double*)M,
                       x, a, b, y);
  return hipGetLastError();
}

hipError_t launch_curl_C(const Grid& g, const double* E, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_curl_C, dim3(nblocks(g.nn, kBlock)), dim3(kBlock), 0, st, g, E, out);
  return hipGetLastError();
}

hipError_t launch_field_op_curl(const Grid& g, const double* E, const double* cC, double ctd2, double* out,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_field_op_curl, dim3(nblocks(g.nn, kBlock)), dim3(kBlock), 0, st, g, E, cC, ctd2, out);
  return hipGetLastError();
}

hipError_t launch_rhs(const Grid& g, const double* E_n, bool jf32, const void* J, const double* BC, double c_j,
                      double c_b, double* b, hipStream_t st) {
  if (jf32)
    hipLaunchKernelGGL(k_rhs<float>, dim3(nblocks(g.nn, kBlock)), dim3(kBlock), 0, st, g, E_n, (const float*)J, BC,
                       c_j, c_b, b);
  else
    hipLaunchKernelGGL(k_rhs<double>, dim3(nblocks(g.nn, kBlock)), dim3(kBlock), 0, st, g, E_n, (const double*)J,
                       BC, c_j, c_b, b);
  return hipGetLastError();
}

hipError_t launch_finish(const Grid& g, const double* E_n, const double* E_t, const double* BC_n,
                         const double* curlC_Et, double ctd, double* E_next, double* BC_next, hipStream_t st) {
  hipLaunchKernelGGL(k_finish, dim3(nblocks(3 * g.nn, kBlock)), dim3(kBlock), 0, st, 3 * g.nn, E_n, E_t, BC_n,
                     curlC_Et, ctd, E_next, BC_next);
  return hipGetLastError();
}

hipError_t launch_centres_to_nodes(const Grid& g, const double* BC, double* BN, float* BN32, hipStream_t st) {
  hipLaunchKernelGGL(k_centres_to_nodes, dim3(nblocks(g.nn, kBlock)), dim3(kBlock), 0, st, g, BC, BN, BN32);
  return hipGetLastError();
}

hipError_t launch_to_f32(int64_t n, const double* src, float* dst, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, st, n, src, dst);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  // a fill kernel rather than a memset node, so the path is safe to capture
  int64_t n = (int64_t)(bytes / 4);
  if (n == 0) return hipSuccess;
  if ((reinterpret_cast<uintptr_t>(p) & 15) == 0 && n >= 4 * kBlock) {
    const int64_t n16 = n / 4;
    const int64_t blocks = std::min<int64_t>(nblocks(n16, kBlock), 8192);
    hipLaunchKernelGGL(k_zero16, dim3(blocks), dim3(kBlock), 0, st, (uint4*)p, n16);
    const int64_t tail = n - 4 * n16;
    if (tail > 0) hipLaunchKernelGGL(k_zero, dim3(1), dim3(kBlock), 0, st, (uint32_t*)p + 4 * n16, tail);
  } else {
    hipLaunchKernelGGL(k_zero, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, st, (uint32_t*)p, n);
  }
  return hipGetLastError();
}

hipError_t launch_take_flag(int* flag, int32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_take_flag, dim3(1), dim3(1), 0, st, flag, out);
  return hipGetLastError();
}

hipError_t launch_dots(const double* V, int64_t ld, int nv, const double* w, int64_t n, double* partial, double* out,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_dots_partial, dim3(kDotBlocks), dim3(kBlock), 0, st, V, ld, nv, w, n, partial);
  hipLaunchKernelGGL(k_dots_final, dim3(nv), dim3(kBlock), 0, st, partial, nv, out);
  return hipGetLastError();
}

hipError_t launch_sub_combo(const double* V, int64_t ld, int nv, const double* coef_host, double* w, int64_t n,
                            hipStream_t st) {
  if (nv < 1 || nv > kMaxRestart + 1) return hipErrorInvalidValue;
  Coefs c;
  for (int v = 0; v < nv; ++v) c.c[v] = coef_host[v];
  hipLaunchKernelGGL(k_sub_combo, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, st, V, ld, nv, c, w, n);
  return hipGetLastError();
}

hipError_t launch_sub_combo_dev(const double* V, int64_t ld, int nv, const double* coef_dev, double* w, int64_t n,
                                hipStream_t st) {
  if (nv < 1) return hipSuccess;
  hipLaunchKernelGGL(k_sub_combo_dev, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, st, V, ld, nv, coef_dev, w, n);
  return hipGetLastError();
}

hipError_t launch_normalize(const double* w, const double* nrm2, double* out, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_normalize, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, st, w, nrm2, out, n);
  return hipGetLastError();
}

hipError_t launch_givens(int j, int m, double* H, double* cs, double* sn, double* gv, const double* h1,
                         const double* h2, const double* hn2, double thresh, int* state, double* hist,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(1), 0, st, j, m, H, cs, sn, gv, h1, h2, hn2, thresh, state, hist);
  return hipGetLastError();
}

hipError_t launch_gmres_start(int m, double beta, double* gv, int* state, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_start, dim3(1), dim3(1), 0, st, m, beta, gv, state);
  return hipGetLastError();
}

hipError_t launch_backsolve(const double* H, const double* gv, int m, int j, double* ny, hipStream_t st) {
  hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(1), 0, st, H, gv, m, j, ny);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, st, n, a, x, b, y);
  return hipGetLastError();
}

hipError_t launch_scale_copy(int64_t n, double a, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_copy, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, st, n, a, x, y);
  return hipGetLastError();
}

hipError_t launch_sumsq(const double* x, int64_t n, double scale, double* partial, double* out, bool accumulate,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq_partial, dim3(kDotBlocks), dim3(kBlock), 0, st, x, n, partial);
  hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(kBlock), 0, st, partial, scale, out, accumulate ? 1 : 0);
  return hipGetLastError();
}

}  // namespace ecsim
