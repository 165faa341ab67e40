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
  // a plane of x or M holds fewer than 2^29 values (checked by the caller),
  // so the per-thread part of every address is a 32-bit byte offset from a
  // uniform base
  const char* xb = (const char*)x;
  const uint32_t own = (uint32_t)gid * (uint32_t)sizeof(TM);
  double y0 = 0.0, y1 = 0.0, y2 = 0.0;
#pragma unroll
  for (int k = 0; k < 14; ++k) {
    int ox, oy, oz;
    offset14(k, ox, oy, oz);
    const char* Mk = (const char*)(M + (int64_t)k * 9 * nn);
    const int64_t pl = nn * (int64_t)sizeof(TM);
    auto mat = [&](int q, uint32_t off) { return (double)*(const TM*)(Mk + q * pl + off); };
    auto xv = [&](int c, uint32_t off) { return *(const double*)(xb + c * nn * 8 + off); };
    {
      const uint32_t gp = (uint32_t)shift(ix, ox, g.nx) +
                          (uint32_t)g.nx * ((uint32_t)shift(iy, oy, g.ny) + (uint32_t)g.ny * (uint32_t)shift(iz, oz, g.nz));
      const double e0 = xv(0, gp * 8u), e1 = xv(1, gp * 8u), e2 = xv(2, gp * 8u);
      y0 = fma(mat(0, own), e0, y0);
      y0 = fma(mat(1, own), e1, y0);
      y0 = fma(mat(2, own), e2, y0);
      y1 = fma(mat(3, own), e0, y1);
      y1 = fma(mat(4, own), e1, y1);
      y1 = fma(mat(5, own), e2, y1);
      y2 = fma(mat(6, own), e0, y2);
      y2 = fma(mat(7, own), e1, y2);
      y2 = fma(mat(8, own), e2, y2);
    }
    if (k > 0) {
      const uint32_t gm = (uint32_t)shift(ix, -ox, g.nx) +
                          (uint32_t)g.nx * ((uint32_t)shift(iy, -oy, g.ny) + (uint32_t)g.ny * (uint32_t)shift(iz, -oz, g.nz));
      const uint32_t gmo = gm * (uint32_t)sizeof(TM);
      const double e0 = xv(0, gm * 8u), e1 = xv(1, gm * 8u), e2 = xv(2, gm * 8u);
      y0 = fma(mat(0, gmo), e0, y0);
      y0 = fma(mat(1, gmo), e1, y0);
      y0 = fma(mat(2, gmo), e2, y0);
      y1 = fma(mat(3, gmo), e0, y1);
      y1 = fma(mat(4, gmo), e1, y1);
      y1 = fma(mat(5, gmo), e2, y1);
      y2 = fma(mat(6, gmo), e0, y2);
      y2 = fma(mat(7, gmo), e1, y2);
      y2 = fma(mat(8, gmo), e2, y2);
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
__device__ __forceinline__ void curl_C_at(const Grid& g, const double* __restrict__ E, int64_t c, double r[3]) {
  const int64_t nn = g.nn;
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
  r[0] = d[1][2] * iy - d[2][1] * iz;
  r[1] = d[2][0] * iz - d[0][2] * ix;
  r[2] = d[0][1] * ix - d[1][0] * iy;
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


// ---------------------------------------------------------------------------
// GMRES kernels (FP64). Each takes one node (its three components) per thread
// in workgroups of kSolveBlock threads, so all of them write and read
// per-workgroup partial sums over the same nblk = ceil(Nn / kSolveBlock)
// slots. A kernel that needs an inner product sums the partials of the kernel
// before it (every workgroup in the same fixed order, so all of them get the
// same value) instead of waiting for a reduction launch of its own.
// ---------------------------------------------------------------------------
constexpr int kVW = kSolveBlock / 64;                 // wavefronts per workgroup
constexpr int kRed = (kMaxRestart + 1) * kVW;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  return v;  // in lane 0
}

// out[v] (LDS) = sum over b < nblk of P[v nblk + b], for v < nv
__device__ void sum_partials(const double* __restrict__ P, int nblk, int nv, double* red, double* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int v = 0; v < nv; ++v) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kSolveBlock) s += P[(int64_t)v * nblk + b];
    s = wave_sum(s);
    if (lane == 0) red[v * kVW + wv] = s;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < nv; v += kSolveBlock) {
    double s = 0.0;
    for (int i = 0; i < kVW; ++i) s += red[v * kVW + i];
    out[v] = s;
  }
  __syncthreads();
}

// P[v nblk + slot] = this workgroup's sum of val(v), for v < nv
template <class F>
__device__ void write_partials(int nv, F val, double* red, double* __restrict__ P, int nblk, int slot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int v = 0; v < nv; ++v) {
    const double s = wave_sum(val(v));
    if (lane == 0) red[v * kVW + wv] = s;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < nv; v += kSolveBlock) {
    double s = 0.0;
    for (int i = 0; i < kVW; ++i) s += red[v * kVW + i];
    P[(int64_t)v * nblk + slot] = s;
  }
}

// Workgroups go to the 8 XCDs in turn; give each XCD a contiguous eighth of
// the nodes, so that the blocks and values read again from a neighbouring
// node are still in that XCD's L2.
__device__ __forceinline__ int xcd_block() {
  int blk = blockIdx.x;
  if ((gridDim.x & 7) == 0) blk = (blk & 7) * (gridDim.x >> 3) + (blk >> 3);
  return blk;
}

// y = (A x)(node) for x = sc X: x + (c theta dt)^2 curl_N curl_C x + cm M x;
// xo = x at the node itself. The curl-curl term is a 27-point stencil over
// the same neighbours the 14 stored mass-matrix blocks couple. It is even in
// the offset o, so it acts on u(o) = x(g + o) + x(g - o) over the 13 stored
// offsets (u(0) = x(g)), and each of its coefficients is an integer weight
// of o times (c theta dt)^2 / (16 h_r h_c) (curl_curl_stencil):
//   (curl_N curl_C x)_r = sum_{c != r} K_rc S_rc - sum_{d != r} K_dd L_dr,
//   S_rc = sum_o o_r o_c (2 - |o_e|) u_c(o)        (e: the third axis),
//   L_dr = sum_o q(o_d) prod_{a != d} (2 - |o_a|) u_r(o),  q(0) = -2, q(+-1) = 1,
// so the weights are compile-time constants and only the six K values are
// read at run time.
// With CURL, d[axis][comp] also collects the edge differences of x over
// cell gid (corners gid + a, a in {0,1}^3, all among the stored offsets):
// curl_C x at that cell is their cross combination.
template <typename TM, bool CURL = false>
__device__ __forceinline__ void apply_at(const Grid& g, const TM* __restrict__ M, const CurlK& K, double cm,
                                         const double* __restrict__ X, double sc, int64_t gid, double y[3],
                                         double xo[3], double (*d)[3] = nullptr) {
  // every plane of X and M holds fewer than 2^29 values (the solver checks),
  // so the per-thread part of an address is a 32-bit byte offset from a
  // uniform base
  const int64_t nn = g.nn;
  int ix, iy, iz;
  decode_cell(g, (int)gid, ix, iy, iz);
  const char* Xb = (const char*)X;
  const uint32_t own = (uint32_t)gid * (uint32_t)sizeof(TM);
  double m0 = 0.0, m1 = 0.0, m2 = 0.0;
  double S[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, L[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int k = 0; k < 14; ++k) {
    int o[3];
    offset14(k, o[0], o[1], o[2]);
    const char* Mk = (const char*)(M + (int64_t)k * 9 * nn);
    const int64_t pl = nn * (int64_t)sizeof(TM);   // bytes per plane of M
    auto mat = [&](int q, uint32_t off) { return (double)*(const TM*)(Mk + q * pl + off); };
    auto xv = [&](int c, uint32_t off) { return sc * *(const double*)(Xb + c * nn * 8 + off); };
    double u[3];
    {
      const uint32_t gp =
          (uint32_t)shift(ix, o[0], g.nx) + (uint32_t)g.nx * ((uint32_t)shift(iy, o[1], g.ny) + (uint32_t)g.ny * (uint32_t)shift(iz, o[2], g.nz));
      const double e0 = xv(0, gp * 8u), e1 = xv(1, gp * 8u), e2 = xv(2, gp * 8u);
      if (k == 0) {
        xo[0] = e0;
        xo[1] = e1;
        xo[2] = e2;
      }
      m0 = fma(mat(0, own), e0, m0);
      m0 = fma(mat(1, own), e1, m0);
      m0 = fma(mat(2, own), e2, m0);
      m1 = fma(mat(3, own), e0, m1);
      m1 = fma(mat(4, own), e1, m1);
      m1 = fma(mat(5, own), e2, m1);
      m2 = fma(mat(6, own), e0, m2);
      m2 = fma(mat(7, own), e1, m2);
      m2 = fma(mat(8, own), e2, m2);
      u[0] = e0;
      u[1] = e1;
      u[2] = e2;
      if (CURL && o[0] >= 0 && o[1] >= 0 && o[2] >= 0) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          d[ax][0] += o[ax] ? e0 : -e0;
          d[ax][1] += o[ax] ? e1 : -e1;
          d[ax][2] += o[ax] ? e2 : -e2;
        }
      }
    }
    if (k > 0) {
      const uint32_t gm = (uint32_t)shift(ix, -o[0], g.nx) +
                          (uint32_t)g.nx * ((uint32_t)shift(iy, -o[1], g.ny) + (uint32_t)g.ny * (uint32_t)shift(iz, -o[2], g.nz));
      const uint32_t gmo = gm * (uint32_t)sizeof(TM);
      const double e0 = xv(0, gm * 8u), e1 = xv(1, gm * 8u), e2 = xv(2, gm * 8u);
      m0 = fma(mat(0, gmo), e0, m0);
      m0 = fma(mat(1, gmo), e1, m0);
      m0 = fma(mat(2, gmo), e2, m0);
      m1 = fma(mat(3, gmo), e0, m1);
      m1 = fma(mat(4, gmo), e1, m1);
      m1 = fma(mat(5, gmo), e2, m1);
      m2 = fma(mat(6, gmo), e0, m2);
      m2 = fma(mat(7, gmo), e1, m2);
      m2 = fma(mat(8, gmo), e2, m2);
      u[0] += e0;
      u[1] += e1;
      u[2] += e2;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (r == c) continue;
        const int e = 3 - r - c;
        const int ws = o[r] * o[c] * (2 - abs(o[e]));
        if (ws != 0) S[r][c] = fma((double)ws, u[c], S[r][c]);
        // L[d = r][comp = c]
        const int wl = (o[r] == 0 ? -2 : 1) * (2 - abs(o[c])) * (2 - abs(o[e]));
        L[r][c] = fma((double)wl, u[c], L[r][c]);
      }
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double cc = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (c != r) cc = fma(K.k[r][c], S[r][c], fma(-K.k[c][c], L[c][r], cc));
    y[r] = xo[r] + cc + cm * (r == 0 ? m0 : (r == 1 ? m1 : m2));
  }
}

__device__ __forceinline__ int* gmres_flags(const GmresState& G) { return (int*)(G.rb + 4 + G.m); }  // 4 ints

// Column j of the Arnoldi process on the device, by one workgroup (every
// thread calls it): H[:, j] from the two Gram-Schmidt passes and the new
// vector's norm hn, the earlier Givens rotations applied to it, a new
// rotation that zeroes H[j+1][j], and the rotated right-hand side g.
// hist[j] = |g[j+1]|, the least-squares residual after j + 1 steps. Once it
// is below the threshold (or the Krylov space broke down) flags[0] = 0, and
// later columns leave everything as it is, so steps launched past
// convergence change nothing. flags[1] = columns that count. The column and
// the rotations are staged in LDS (sh: 3 kMaxRestart + 2 doubles), so the
// serial part runs on LDS values.
__device__ void givens_column(int j, const GmresState& G, double hn, double* sh) {
  int* fl = gmres_flags(G);
  double* col = sh;                        // j + 2
  double* c = sh + kMaxRestart + 2;        // j
  double* sn = c + kMaxRestart;            // j
  const int t = threadIdx.x, m = G.m;
  const bool active = fl[0] != 0;
  if (active) {
    if (t <= j) col[t] = G.h1[t] + G.h2[t];
    if (t < j) {
      c[t] = G.cs[t];
      sn[t] = G.sn[t];
    }
  }
  __syncthreads();
  if (t == 0) {
    double* hist = G.rb + 4;
    if (!active) {
      hist[j] = -1.0;
    } else {
      col[j + 1] = hn;
      for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = c[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + c[i] * b;
      }
      const double a = col[j], b = col[j + 1];
      const double rr = hypot(a, b);
      const double cj = rr > 0.0 ? a / rr : 1.0, sj = rr > 0.0 ? b / rr : 0.0;
      col[j] = rr;
      col[j + 1] = 0.0;
      G.cs[j] = cj;
      G.sn[j] = sj;
      const double gj = G.gv[j];
      G.gv[j + 1] = -sj * gj;
      G.gv[j] = cj * gj;
      hist[j] = fabs(sj * gj);
      fl[1] = j + 1;
      if (hist[j] <= G.rb[0] || hn == 0.0) fl[0] = 0;
    }
  }
  __syncthreads();
  if (active && t <= j + 1) G.H[(int64_t)t * m + j] = col[t];
}

// R = b - A X and the partial |R|^2 into Pr. FIRST: X = E^n, and b =
// E^n + c_j J + c_b curl_N(B_C^n) is formed here (written to bout, with
// its partial |b|^2 into Pb = Pr - nblk) and E_theta = E^n. LAST (X =
// E^{n+theta}, the end of a batch): also the field advance
// E^{n+1} = 2 E^{n+theta} - E^n, B_C^{n+1} = 2 (B_C^n - ctd curl_C E^{n+theta}) - B_C^n
// (cell gid's curl from the neighbours the operator loads), and yp = yn,
// the update X now holds.
struct ResidualArgs {
  const double* X;
  const double* b;
  double* R;
  double* Pr;
  // FIRST
  const void* J;
  const double* BC;
  double c_j, c_b;
  double* bout;
  double* Et;
  // LAST
  const double* En;
  double ctd;
  double* En1;
  double* BCn1;
};
template <typename TM, bool FIRST, bool LAST>
__global__ void __launch_bounds__(kSolveBlock) k_residual_op(Grid g, const TM* __restrict__ M, CurlK K, double cm,
                                                             ResidualArgs A, int nblk, GmresState G) {
  __shared__ double red[2 * kVW];
  if (LAST && blockIdx.x == 0 && threadIdx.x == 0) {
    int* fl = gmres_flags(G);
    for (int v = 0; v < fl[3]; ++v) G.yp[v] = G.yn[v];
    fl[2] = fl[3];
  }
  const int blk = xcd_block();
  const int64_t nn = g.nn, i = (int64_t)blk * kSolveBlock + threadIdx.x;
  double r[3] = {0.0, 0.0, 0.0}, bv[3] = {0.0, 0.0, 0.0};
  if (i < nn) {
    if (FIRST) {
      double cn[3];
      curl_N_at(g, A.BC, i, cn);
      const TM* J = (const TM*)A.J;
      for (int c = 0; c < 3; ++c) {
        const double e = A.X[c * nn + i];
        bv[c] = (e + A.c_j * (double)J[c * nn + i]) + A.c_b * cn[c];
        A.bout[c * nn + i] = bv[c];
        A.Et[c * nn + i] = e;
      }
      // keep the right-hand side's loads out of the operator's schedule
      __builtin_amdgcn_sched_barrier(0);
    }
    double y[3], xo[3], d[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    apply_at<TM, LAST>(g, M, K, cm, A.X, 1.0, i, y, xo, d);
    if (LAST) __builtin_amdgcn_sched_barrier(0);
    if (!FIRST)
      for (int c = 0; c < 3; ++c) bv[c] = A.b[c * nn + i];
    for (int c = 0; c < 3; ++c) {
      r[c] = bv[c] - y[c];
      A.R[c * nn + i] = r[c];
    }
    if (LAST) {
      const double ix = 1.0 / (4.0 * g.hx), iy = 1.0 / (4.0 * g.hy), iz = 1.0 / (4.0 * g.hz);
      const double cc[3] = {d[1][2] * iy - d[2][1] * iz, d[2][0] * iz - d[0][2] * ix, d[0][1] * ix - d[1][0] * iy};
      for (int c = 0; c < 3; ++c) {
        const double en = A.En[c * nn + i], bc = A.BC[c * nn + i];
        A.En1[c * nn + i] = 2.0 * xo[c] - en;
        A.BCn1[c * nn + i] = 2.0 * (bc - A.ctd * cc[c]) - bc;
      }
    }
  }
  if (FIRST)
    write_partials(
        2, [&](int v) { return v == 0 ? bv[0] * bv[0] + bv[1] * bv[1] + bv[2] * bv[2] : r[0] * r[0] + r[1] * r[1] + r[2] * r[2]; },
        red, A.Pr - nblk, nblk, blk);
  else
    write_partials(1, [&](int) { return r[0] * r[0] + r[1] * r[1] + r[2] * r[2]; }, red, A.Pr, nblk, blk);
}

// Step s of the Arnoldi process, first kernel: V_s = w_s / |w_s| (|w_s|^2
// from the partials P3), w = A V_s into Wout and the first Gram-Schmidt
// pass's partial inner products <V_v, w>, v <= s, into P1. Workgroup 0 also
// starts the restart cycle (s = 0: g = (beta, 0, ...), the threshold from
// |b|) or closes column s - 1 (its Givens rotation needs |w_s|).
template <typename TM>
__global__ void __launch_bounds__(kSolveBlock) k_arnoldi_op(Grid g, const TM* __restrict__ M, CurlK K,
                                                            double cm, const double* __restrict__ Win,
                                                            double* __restrict__ Wout, double* __restrict__ V,
                                                            int64_t ld, int s, int mode,
                                                            const double* __restrict__ P3, double* __restrict__ P1,
                                                            int nblk, GmresState G) {
  __shared__ double red[kRed];
  __shared__ double sc[2];
  sum_partials(P3, nblk, 1, red, sc);
  const double hn = sqrt(sc[0]);
  const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
  __shared__ double gsh[3 * kMaxRestart + 2];
  if (blockIdx.x == 0 && mode == kArnoldiGivens) givens_column(s - 1, G, hn, gsh);
  if (blockIdx.x == 0 && mode == kArnoldiStart) {
    sum_partials(G.Pb, nblk, 1, red, sc + 1);
    if (threadIdx.x == 0) {
      {
        const double thresh = 0.5 * G.tol * sqrt(sc[1]);
        G.rb[0] = thresh;
        G.rb[1] = hn;
        for (int i = 0; i <= G.m; ++i) G.gv[i] = i == 0 ? hn : 0.0;
        int* fl = gmres_flags(G);
        fl[0] = hn > thresh ? 1 : 0;
        fl[1] = 0;
        fl[2] = 0;
        fl[3] = 0;
      }
    }
  }
  const int blk = xcd_block();
  const int64_t nn = g.nn, i = (int64_t)blk * kSolveBlock + threadIdx.x;
  const bool live = i < nn;
  double y[3] = {0.0, 0.0, 0.0}, xo[3] = {0.0, 0.0, 0.0};
  if (live) {
    apply_at(g, M, K, cm, Win, inv, i, y, xo);
    double* Vs = V + (int64_t)s * ld;
    for (int c = 0; c < 3; ++c) {
      Vs[c * nn + i] = xo[c];
      Wout[c * nn + i] = y[c];
    }
  }
  write_partials(
      s + 1,
      [&](int v) {
        if (!live) return 0.0;
        if (v == s) return xo[0] * y[0] + xo[1] * y[1] + xo[2] * y[2];
        const double* Vv = V + (int64_t)v * ld;
        return Vv[i] * y[0] + Vv[nn + i] * y[1] + Vv[2 * nn + i] * y[2];
      },
      red, P1, nblk, blk);
}

// A Gram-Schmidt pass over V_0..V_{k-1}: h_v = the sums of the partials Pin,
// w -= sum_v h_v V_v, then either the next pass's partial inner products
// <V_v, w> (NORM false) or the partial |w|^2 (NORM true) into Pout.
// Workgroup 0 stores h into coef for the Givens update. w and the first kKV
// basis vectors are loaded before the partials are summed, so their latency
// overlaps the reduction.
constexpr int kKV = 8;
template <bool NORM>
__global__ void __launch_bounds__(kSolveBlock) k_cgs_pass(const double* __restrict__ V, int64_t ld, int k, int64_t nn,
                                                          const double* __restrict__ Pin, double* __restrict__ coef,
                                                          double* __restrict__ W, double* __restrict__ Pout,
                                                          int nblk) {
  __shared__ double red[kRed];
  __shared__ double h[kMaxRestart + 1];
  const int64_t i = (int64_t)blockIdx.x * kSolveBlock + threadIdx.x;
  const bool live = i < nn;
  double w[3] = {0.0, 0.0, 0.0}, vr[kKV][3];
#pragma unroll
  for (int v = 0; v < kKV; ++v) vr[v][0] = vr[v][1] = vr[v][2] = 0.0;
  if (live) {
    for (int c = 0; c < 3; ++c) w[c] = W[c * nn + i];
#pragma unroll
    for (int v = 0; v < kKV; ++v)
      if (v < k)
        for (int c = 0; c < 3; ++c) vr[v][c] = V[(int64_t)v * ld + c * nn + i];
  }
  sum_partials(Pin, nblk, k, red, h);
  if (blockIdx.x == 0)
    for (int v = threadIdx.x; v < k; v += kSolveBlock) coef[v] = h[v];
  if (live) {
#pragma unroll
    for (int v = 0; v < kKV; ++v)
      if (v < k)
        for (int c = 0; c < 3; ++c) w[c] = fma(-h[v], vr[v][c], w[c]);
    for (int v = kKV; v < k; ++v) {
      const double* Vv = V + (int64_t)v * ld;
      for (int c = 0; c < 3; ++c) w[c] = fma(-h[v], Vv[c * nn + i], w[c]);
    }
    for (int c = 0; c < 3; ++c) W[c * nn + i] = w[c];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (NORM) {
    const double sq = wave_sum(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (lane == 0) red[wv] = sq;
  } else {
#pragma unroll
    for (int v = 0; v < kKV; ++v)
      if (v < k) {
        const double d = wave_sum(vr[v][0] * w[0] + vr[v][1] * w[1] + vr[v][2] * w[2]);
        if (lane == 0) red[v * kVW + wv] = d;
      }
    for (int v = kKV; v < k; ++v) {
      const double* Vv = V + (int64_t)v * ld;
      const double d = wave_sum(live ? Vv[i] * w[0] + Vv[nn + i] * w[1] + Vv[2 * nn + i] * w[2] : 0.0);
      if (lane == 0) red[v * kVW + wv] = d;
    }
  }
  __syncthreads();
  const int nv = NORM ? 1 : k;
  for (int v = threadIdx.x; v < nv; v += kSolveBlock) {
    double t = 0.0;
    for (int q = 0; q < kVW; ++q) t += red[v * kVW + q];
    Pout[(int64_t)v * nblk + blockIdx.x] = t;
  }
}

// After the last step of a batch: the Givens update of column j, then y
// from the upper triangle H y = g over the columns that count (flags[1]),
// into yn (flags[3] = their number). The triangle is staged in LDS when it
// has at most kTri columns.
constexpr int kTri = 40;
__global__ void __launch_bounds__(kSolveBlock) k_givens_tail(int j, const double* __restrict__ P3, int nblk,
                                                             GmresState G) {
  __shared__ double red[kVW];
  __shared__ double sc[1];
  __shared__ double gsh[3 * kMaxRestart + 2];
  __shared__ double tri[kTri * (kTri + 1) / 2 + kTri];
  __shared__ double yl[kTri];
  __shared__ int cols;
  sum_partials(P3, nblk, 1, red, sc);
  givens_column(j, G, sqrt(sc[0]), gsh);
  int* fl = gmres_flags(G);
  if (threadIdx.x == 0) cols = fl[1];   // written by this thread in givens_column
  __syncthreads();
  const int m = G.m, jj = cols;
  if (jj <= kTri) {
    // row i of the triangle (columns i..jj-1) at tri[i jj - i (i - 1) / 2 ...], then g
    for (int e = threadIdx.x; e < jj * (jj + 1) / 2; e += kSolveBlock) {
      int i = 0, r = e;
      while (r >= jj - i) {
        r -= jj - i;
        ++i;
      }
      tri[e] = G.H[(int64_t)i * m + i + r];
    }
    for (int e = threadIdx.x; e < jj; e += kSolveBlock) tri[jj * (jj + 1) / 2 + e] = G.gv[e];
    __syncthreads();
    if (threadIdx.x == 0) {
      const double* gg = tri + jj * (jj + 1) / 2;
      for (int i = jj - 1; i >= 0; --i) {
        const double* row = tri + i * jj - i * (i - 1) / 2;   // row[k - i] = H[i][k]
        double s = gg[i];
        for (int k = i + 1; k < jj; ++k) s -= row[k - i] * yl[k];
        yl[i] = s / row[0];
        G.yn[i] = yl[i];
      }
      fl[3] = jj;
    }
  } else if (threadIdx.x == 0) {
    for (int i = jj - 1; i >= 0; --i) {
      double s = G.gv[i];
      for (int k = i + 1; k < jj; ++k) s -= G.H[(int64_t)i * m + k] * G.yn[k];
      G.yn[i] = s / G.H[(int64_t)i * m + i];
    }
    fl[3] = jj;
  }
}

// X += V (yn - yp): the cycle's update so far is V yp (flags[2] columns),
// the one wanted is V yn (flags[3] columns)
__global__ void __launch_bounds__(kSolveBlock) k_update_x(const double* __restrict__ V, int64_t ld, int64_t nn,
                                                          double* __restrict__ X, GmresState G) {
  __shared__ double d[kMaxRestart];
  const int* fl = gmres_flags(G);
  const int jn = fl[3], jp = fl[2], j = jn > jp ? jn : jp;
  for (int v = threadIdx.x; v < j; v += kSolveBlock) d[v] = (v < jn ? G.yn[v] : 0.0) - (v < jp ? G.yp[v] : 0.0);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kSolveBlock + threadIdx.x;
  if (i >= nn) return;
  for (int c = 0; c < 3; ++c) {
    double x = X[c * nn + i];
    for (int v = 0; v < j; ++v) x = fma(d[v], V[(int64_t)v * ld + c * nn + i], x);
    X[c * nn + i] = x;
  }
}

// E^{n+1} = 2 E^{n+theta} - E^n; B^{n+1} = 2 (B^n - ctd curl_C E^{n+theta}) - B^n
// and, with G.m > 0, yp = yn: the update now in X
__global__ void __launch_bounds__(kBlock) k_finish(Grid g, const double* __restrict__ En,
                                                   const double* __restrict__ Et, const double* __restrict__ BCn,
                                                   double ctd, double* __restrict__ En1, double* __restrict__ BCn1,
                                                   GmresState G) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && G.m > 0) {
    int* fl = gmres_flags(G);
    for (int v = 0; v < fl[3]; ++v) G.yp[v] = G.yn[v];
    fl[2] = fl[3];
  }
  const int64_t nn = g.nn, c = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (c >= nn) return;
  double cc[3];
  curl_C_at(g, Et, c, cc);
  for (int comp = 0; comp < 3; ++comp) {
    const int64_t i = comp * nn + c;
    En1[i] = 2.0 * Et[i] - En[i];
    const double bt = BCn[i] - ctd * cc[comp];
    BCn1[i] = 2.0 * bt - BCn[i];
  }
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

// ---------------------------------------------------------------------------
// GMRES launchers
// ---------------------------------------------------------------------------
void curl_curl_stencil(const Grid& g, double ctd2, CurlK& K) {
  // curl_C and curl_N each weigh a difference along axis d by 1 / (4 h_d)
  const double ih[3] = {1.0 / (4.0 * g.hx), 1.0 / (4.0 * g.hy), 1.0 / (4.0 * g.hz)};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) K.k[r][c] = ctd2 * ih[r] * ih[c];
}

int solve_blocks(const Grid& g) { return (int)((g.nn + kSolveBlock - 1) / kSolveBlock); }

hipError_t launch_residual_first(const Grid& g, bool mf32, const void* M, const CurlK& K, double cm,
                                 const double* E_n, const void* J, const double* BC, double c_j, double c_b,
                                 double* b, double* E_t, double* R, double* Pb, double* Pr, hipStream_t st) {
  const int nb = solve_blocks(g);
  if (Pr != Pb + nb) return hipErrorInvalidValue;
  ResidualArgs A{};
  A.X = E_n;
  A.R = R;
  A.Pr = Pr;
  A.J = J;
  A.BC = BC;
  A.c_j = c_j;
  A.c_b = c_b;
  A.bout = b;
  A.Et = E_t;
  GmresState none{};
  if (mf32)
    hipLaunchKernelGGL((k_residual_op<float, true, false>), dim3(nb), dim3(kSolveBlock), 0, st, g, (const float*)M,
                       K, cm, A, nb, none);
  else
    hipLaunchKernelGGL((k_residual_op<double, true, false>), dim3(nb), dim3(kSolveBlock), 0, st, g,
                       (const double*)M, K, cm, A, nb, none);
  return hipGetLastError();
}

hipError_t launch_residual_last(const Grid& g, bool mf32, const void* M, const CurlK& K, double cm,
                                const double* E_t, const double* b, double* R, double* Pr, const double* E_n,
                                const double* BC_n, double ctd, double* E_next, double* BC_next,
                                const GmresState& G, hipStream_t st) {
  const int nb = solve_blocks(g);
  ResidualArgs A{};
  A.X = E_t;
  A.b = b;
  A.R = R;
  A.Pr = Pr;
  A.BC = BC_n;
  A.En = E_n;
  A.ctd = ctd;
  A.En1 = E_next;
  A.BCn1 = BC_next;
  if (mf32)
    hipLaunchKernelGGL((k_residual_op<float, false, true>), dim3(nb), dim3(kSolveBlock), 0, st, g, (const float*)M,
                       K, cm, A, nb, G);
  else
    hipLaunchKernelGGL((k_residual_op<double, false, true>), dim3(nb), dim3(kSolveBlock), 0, st, g,
                       (const double*)M, K, cm, A, nb, G);
  return hipGetLastError();
}

hipError_t launch_arnoldi_op(const Grid& g, bool mf32, const void* M, const CurlK& K, double cm,
                             const double* Win, double* Wout, double* V, int64_t ld, int s, int mode,
                             const double* P3, double* P1, const GmresState& G, hipStream_t st) {
  if (s < 0 || s >= G.m) return hipErrorInvalidValue;
  const int nb = solve_blocks(g);
  if (mf32)
    hipLaunchKernelGGL(k_arnoldi_op<float>, dim3(nb), dim3(kSolveBlock), 0, st, g, (const float*)M, K, cm, Win,
                       Wout, V, ld, s, mode, P3, P1, nb, G);
  else
    hipLaunchKernelGGL(k_arnoldi_op<double>, dim3(nb), dim3(kSolveBlock), 0, st, g, (const double*)M, K, cm,
                       Win, Wout, V, ld, s, mode, P3, P1, nb, G);
  return hipGetLastError();
}

hipError_t launch_cgs_pass(const Grid& g, bool norm, const double* V, int64_t ld, int k, const double* Pin,
                           double* coef, double* W, double* Pout, hipStream_t st) {
  if (k < 1 || k > kMaxRestart) return hipErrorInvalidValue;
  const int nb = solve_blocks(g);
  if (norm)
    hipLaunchKernelGGL(k_cgs_pass<true>, dim3(nb), dim3(kSolveBlock), 0, st, V, ld, k, g.nn, Pin, coef, W, Pout, nb);
  else
    hipLaunchKernelGGL(k_cgs_pass<false>, dim3(nb), dim3(kSolveBlock), 0, st, V, ld, k, g.nn, Pin, coef, W, Pout, nb);
  return hipGetLastError();
}

hipError_t launch_givens_tail(const Grid& g, int j, const double* P3, const GmresState& G, hipStream_t st) {
  if (j < 0 || j >= G.m) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_givens_tail, dim3(1), dim3(kSolveBlock), 0, st, j, P3, solve_blocks(g), G);
  return hipGetLastError();
}

hipError_t launch_update_x(const Grid& g, const double* V, int64_t ld, double* X, const GmresState& G,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_update_x, dim3(solve_blocks(g)), dim3(kSolveBlock), 0, st, V, ld, g.nn, X, G);
  return hipGetLastError();
}

hipError_t launch_finish(const Grid& g, const double* E_n, const double* E_t, const double* BC_n, double ctd,
                         double* E_next, double* BC_next, const GmresState* G, hipStream_t st) {
  GmresState none{};
  hipLaunchKernelGGL(k_finish, dim3(nblocks(g.nn, kBlock)), dim3(kBlock), 0, st, g, E_n, E_t, BC_n, ctd, E_next,
                     BC_next, G ? *G : none);
  return hipGetLastError();
}

hipError_t launch_sumsq(const double* x, int64_t n, double scale, double* partial, double* out, bool accumulate,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq_partial, dim3(kDotBlocks), dim3(kBlock), 0, st, x, n, partial);
  hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(kBlock), 0, st, partial, scale, out, accumulate ? 1 : 0);
  return hipGetLastError();
}

}  // namespace ecsim
