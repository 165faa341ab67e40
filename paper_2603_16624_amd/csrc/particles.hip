// Particle kernels: mover (Eqs. 4, 5, 8), per-particle atomic moment deposit
// (Eqs. 1, 3) for particles in any order, and the per-species counting sort.
#include <algorithm>
#include "internal.h"

namespace ecsim {

namespace {

constexpr int kBlock = 256;

// Particle state access for both storage forms.
template <typename T, bool CELL>
struct PState;

template <>
struct PState<double, false> {
  __device__ __forceinline__ static Stencil<double> stencil(const Grid& g, const double* p0, const double* p1,
                                                           const double* p2, const int32_t*, int p) {
    return stencil_abs(g, p0[p], p1[p], p2[p]);
  }
};

template <>
struct PState<float, true> {
  __device__ __forceinline__ static Stencil<float> stencil(const Grid& g, const float* p0, const float* p1,
                                                          const float* p2, const int32_t* cell, int p) {
    return stencil_cell(g, cell[p], p0[p], p1[p], p2[p]);
  }
};

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) s += red[i];
  return s;
}

// ---------------------------------------------------------------------------
// mover
// ---------------------------------------------------------------------------
template <typename T, bool CELL>
__global__ void __launch_bounds__(kBlock) k_move(Grid g, int np, T* __restrict__ p0, T* __restrict__ p1,
                                                 T* __restrict__ p2, int32_t* __restrict__ cell,
                                                 T* __restrict__ v0, T* __restrict__ v1, T* __restrict__ v2,
                                                 const T* __restrict__ E, const T* __restrict__ B, T beta,
                                                 T dth0, T dth1, T dth2, const T* __restrict__ q,
                                                 double q_const, double inv_qom, double* ke) {
  double kel = 0.0;
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < np; p += gridDim.x * kBlock) {
    Stencil<T> s = PState<T, CELL>::stencil(g, p0, p1, p2, cell, p);
    T W[8];
    int64_t nd[8];
    corners(g, s, W, nd);
    Vec3<T> Ep = gather(E, g.nn, W, nd);
    Vec3<T> Bp = gather(B, g.nn, W, nd);
    Vec3<T> vn = advance_velocity(Bp, beta, Vec3<T>{v0[p], v1[p], v2[p]}, Ep);
    note_nonfinite(g, !(finite(vn.x) && finite(vn.y) && finite(vn.z)));
    v0[p] = vn.x;
    v1[p] = vn.y;
    v2[p] = vn.z;
    if constexpr (CELL) {
      int ix = s.i[0], iy = s.i[1], iz = s.i[2];
      float ox = push_offset(s.w1[0], vn.x, dth0, ix, g.nx);
      float oy = push_offset(s.w1[1], vn.y, dth1, iy, g.ny);
      float oz = push_offset(s.w1[2], vn.z, dth2, iz, g.nz);
      p0[p] = ox;
      p1[p] = oy;
      p2[p] = oz;
      cell[p] = ix + g.nx * (iy + g.ny * iz);
    } else {
      p0[p] = push_abs(p0[p], g.pdt[0], vn.x, g.nx * g.hx);
      p1[p] = push_abs(p1[p], g.pdt[1], vn.y, g.ny * g.hy);
      p2[p] = push_abs(p2[p], g.pdt[2], vn.z, g.nz * g.hz);
    }
    if (ke) {
      double qp = q ? (double)q[p] : q_const;
      double vx = vn.x, vy = vn.y, vz = vn.z;
      kel += 0.5 * (qp * inv_qom) * ((vx * vx + vy * vy) + vz * vz);
    }
  }
  if (ke) {
    double s = block_sum(kel);
    if (threadIdx.x == 0) unsafeAtomicAdd(ke, s);
  }
}

// ---------------------------------------------------------------------------
// per-particle atomic deposit (any particle order)
// ---------------------------------------------------------------------------
template <typename T, bool CELL>
__global__ void __launch_bounds__(kBlock) k_deposit_atomic(Grid g, int np, const T* __restrict__ p0,
                                                           const T* __restrict__ p1, const T* __restrict__ p2,
                                                           const int32_t* __restrict__ cell,
                                                           const T* __restrict__ v0, const T* __restrict__ v1,
                                                           const T* __restrict__ v2, const T* __restrict__ q,
                                                           T q_const, T beta, const T* __restrict__ B,
                                                           T* __restrict__ J, T* __restrict__ M) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= np) return;
  Stencil<T> s = PState<T, CELL>::stencil(g, p0, p1, p2, cell, p);
  T W[8];
  int64_t nd[8];
  corners(g, s, W, nd);
  Vec3<T> Bp = gather(B, g.nn, W, nd);
  T a[9];
  rotation(Bp, beta, a);
  Vec3<T> vh = matvec(a, Vec3<T>{v0[p], v1[p], v2[p]});
  const T qp = q ? q[p] : q_const;
  const T V = T(g.V);
  const T cj = qp / V;
  const T cm = (qp * beta) / V;
  const int64_t nn = g.nn;
  note_nonfinite(g, !(finite(vh.x) && finite(vh.y) && finite(vh.z) && finite(cj) && finite(cm) && finite(W[0]) &&
                      finite(W[7])));
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    T w = cj * W[c];
    unsafeAtomicAdd(&J[nd[c]], w * vh.x);
    unsafeAtomicAdd(&J[nn + nd[c]], w * vh.y);
    unsafeAtomicAdd(&J[2 * nn + nd[c]], w * vh.z);
  }
  for (int ca = 0; ca < 8; ++ca) {
    for (int cb = ca; cb < 8; ++cb) {
      bool at_a;
      int k = pair_block(ca, cb, at_a);
      int64_t node = at_a ? nd[ca] : nd[cb];
      T w = (cm * W[ca]) * W[cb];
      T* Mk = M + (int64_t)k * 9 * nn + node;
#pragma unroll
      for (int ij = 0; ij < 9; ++ij) unsafeAtomicAdd(&Mk[ij * nn], w * a[ij]);
    }
  }
}

// ---------------------------------------------------------------------------
// diagnostic moments, any particle order (Sec. III, diagnostics for I/O):
// rho += q W / V, Jd += q v W / V, P_ij += q v_i v_j W / V (xx xy xz yy yz zz)
// ---------------------------------------------------------------------------
// (TA: the accumulator type; the FP32 form accumulates in FP64, since a node
// takes thousands of mixed-sign terms in no particular order)
template <typename T, bool CELL, typename TA>
__global__ void __launch_bounds__(kBlock) k_diag_atomic(Grid g, int np, const T* __restrict__ p0,
                                                        const T* __restrict__ p1, const T* __restrict__ p2,
                                                        const int32_t* __restrict__ cell, const T* __restrict__ v0,
                                                        const T* __restrict__ v1, const T* __restrict__ v2,
                                                        const T* __restrict__ q, T q_const, TA* __restrict__ rho,
                                                        TA* __restrict__ Jd, TA* __restrict__ P) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= np) return;
  Stencil<T> s = PState<T, CELL>::stencil(g, p0, p1, p2, cell, p);
  T W[8];
  int64_t nd[8];
  corners(g, s, W, nd);
  const T c = (q ? q[p] : q_const) / T(g.V);
  const T vx = v0[p], vy = v1[p], vz = v2[p];
  const T f[10] = {c, c * vx, c * vy, c * vz, (c * vx) * vx, (c * vx) * vy, (c * vx) * vz,
                   (c * vy) * vy, (c * vy) * vz, (c * vz) * vz};
  note_nonfinite(g, !(finite(f[4]) && finite(f[7]) && finite(f[9]) && finite(W[0]) && finite(W[7])));
  const int64_t nn = g.nn;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    unsafeAtomicAdd(&rho[nd[a]], (TA)(f[0] * W[a]));
#pragma unroll
    for (int k = 0; k < 3; ++k) unsafeAtomicAdd(&Jd[k * nn + nd[a]], (TA)(f[1 + k] * W[a]));
#pragma unroll
    for (int k = 0; k < 6; ++k) unsafeAtomicAdd(&P[k * nn + nd[a]], (TA)(f[4 + k] * W[a]));
  }
}

// out += (float)acc over n entries
__global__ void __launch_bounds__(kBlock) k_add_rounded(int64_t n, const double* __restrict__ acc,
                                                        float* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    out[i] += (float)acc[i];
}

// ---------------------------------------------------------------------------
// counting sort by cell
// ---------------------------------------------------------------------------
template <typename T, bool CELL>
__device__ __forceinline__ int particle_key(const Grid& g, const T* p0, const T* p1, const T* p2,
                                            const int32_t* cell, int p) {
  if constexpr (CELL) {
    return cell[p];
  } else {
    Stencil<double> s = stencil_abs(g, p0[p], p1[p], p2[p]);
    return s.i[0] + g.nx * (s.i[1] + g.ny * s.i[2]);
  }
}

template <typename T, bool CELL>
__global__ void __launch_bounds__(kBlock) k_sort_count(Grid g, int np, const T* __restrict__ p0,
                                                       const T* __restrict__ p1, const T* __restrict__ p2,
                                                       const int32_t* __restrict__ cell, int* __restrict__ counts,
                                                       int* __restrict__ keys, int* __restrict__ ranks) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  const bool active = p < np;
  int key = active ? particle_key<T, CELL>(g, p0, p1, p2, cell, p) : -1;
  // wave-aggregated atomics: one atomic per distinct key in the wavefront
  unsigned long long pending = __ballot(active);
  const int lane = threadIdx.x & 63;
  int my_rank = 0;
  while (pending) {
    int leader = __ffsll((unsigned long long)pending) - 1;
    int lkey = __shfl(key, leader);
    unsigned long long grp = __ballot(key == lkey) & pending;
    int base = 0;
    if (lane == leader) base = atomicAdd(&counts[lkey], __popcll(grp));
    base = __shfl(base, leader);
    if ((grp >> lane) & 1ull) my_rank = base + __popcll(grp & ((1ull << lane) - 1ull));
    pending &= ~grp;
  }
  if (active) {
    keys[p] = key;
    ranks[p] = my_rank;
  }
}

constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

// exclusive scan of one tile in LDS; returns the tile total
__device__ int block_exclusive_scan(int* vals /* kScanItems per thread, in/out */) {
  __shared__ int sh[kScanBlock];
  int t = 0;
  for (int i = 0; i < kScanItems; ++i) t += vals[i];
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int x = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += x;
    __syncthreads();
  }
  int incl = sh[threadIdx.x];
  int total = sh[kScanBlock - 1];
  int run = incl - t;
  for (int i = 0; i < kScanItems; ++i) {
    int v = vals[i];
    vals[i] = run;
    run += v;
  }
  __syncthreads();
  return total;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_tiles(const int* __restrict__ in, int n, int* __restrict__ out,
                                                           int* __restrict__ tile_sums) {
  int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  for (int i = 0; i < kScanItems; ++i) v[i] = (base + i < n) ? in[base + i] : 0;
  int total = block_exclusive_scan(v);
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) out[base + i] = v[i];
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// single block: exclusive scan of the tile sums (ntiles <= kScanTile)
__global__ void __launch_bounds__(kScanBlock) k_scan_sums(int* __restrict__ sums, int ntiles, int* __restrict__ total) {
  int base = threadIdx.x * kScanItems;
  int v[kScanItems];
  for (int i = 0; i < kScanItems; ++i) v[i] = (base + i < ntiles) ? sums[base + i] : 0;
  int t = block_exclusive_scan(v);
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < ntiles) sums[base + i] = v[i];
  if (threadIdx.x == 0) *total = t;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_add(int* __restrict__ out, int n, const int* __restrict__ sums,
                                                         const int* __restrict__ total_src) {
  int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int add = sums[blockIdx.x];
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) out[base + i] += add;
  // a scan over more than one level of tiles: the total comes from the level above
  if (total_src && blockIdx.x == 0 && threadIdx.x == 0) out[n] = *total_src;
}

template <typename T, bool CELL>
__global__ void __launch_bounds__(kBlock) k_sort_scatter(
    int np, const int* __restrict__ keys, const int* __restrict__ ranks, const int* __restrict__ start,
    const T* __restrict__ s0, const T* __restrict__ s1, const T* __restrict__ s2, const int32_t* __restrict__ sc,
    const T* __restrict__ u0, const T* __restrict__ u1, const T* __restrict__ u2, const T* __restrict__ sq,
    T* __restrict__ d0, T* __restrict__ d1, T* __restrict__ d2, int32_t* __restrict__ dc, T* __restrict__ w0,
    T* __restrict__ w1, T* __restrict__ w2, T* __restrict__ dq, int32_t* __restrict__ perm) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= np) return;
  int d = start[keys[p]] + ranks[p];
  d0[d] = s0[p];
  d1[d] = s1[p];
  d2[d] = s2[p];
  if constexpr (CELL) dc[d] = sc[p];
  w0[d] = u0[p];
  w1[d] = u1[p];
  w2[d] = u2[p];
  if (sq) dq[d] = sq[p];
  if (perm) perm[d] = p;
}

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
// grid-stride kernels: enough blocks to fill 256 CUs several times over
inline unsigned nblocks_capped(int64_t n, int b) {
  unsigned nb = nblocks(n, b);
  return nb < 4096u ? nb : 4096u;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_move(const Grid& g, bool f32, const SpeciesArgs& sp, const void* E, const void* B, double* ke,
                       hipStream_t st) {
  if (sp.np == 0) return hipSuccess;
  const double beta = sp.qom * g.dt / 2.0;
  const double inv_qom = 1.0 / integrated_qom(sp.qom, g.dt, f32);
  if (f32) {
    hipLaunchKernelGGL((k_move<float, true>), dim3(nblocks_capped(sp.np, kBlock)), dim3(kBlock), 0, st, g, sp.np,
                       (float*)sp.pos[0], (float*)sp.pos[1], (float*)sp.pos[2], sp.cell, (float*)sp.vel[0],
                       (float*)sp.vel[1], (float*)sp.vel[2], (const float*)E, (const float*)B, (float)beta,
                       (float)(g.pdt[0] / g.hx), (float)(g.pdt[1] / g.hy), (float)(g.pdt[2] / g.hz), (const float*)sp.q,
                       sp.q_const, inv_qom, ke);
  } else {
    hipLaunchKernelGGL((k_move<double, false>), dim3(nblocks_capped(sp.np, kBlock)), dim3(kBlock), 0, st, g, sp.np,
                       (double*)sp.pos[0], (double*)sp.pos[1], (double*)sp.pos[2], (int32_t*)nullptr,
                       (double*)sp.vel[0], (double*)sp.vel[1], (double*)sp.vel[2], (const double*)E,
                       (const double*)B, beta, 0.0, 0.0, 0.0, (const double*)sp.q, sp.q_const, inv_qom, ke);
  }
  return hipGetLastError();
}

hipError_t launch_diagnostics_atomic(const Grid& g, bool f32, const SpeciesArgs* sp, int ns, void* rho, void* Jd,
                                     void* P, void* acc, hipStream_t st) {
  const int64_t nn = g.nn;
  hipError_t e;
  double* const a = (double*)acc;   // FP32 form: [10][Nn] FP64 accumulators
  if (f32 && (e = launch_zero(a, sizeof(double) * 10 * (size_t)nn, st)) != hipSuccess) return e;
  for (int s = 0; s < ns; ++s) {
    if (sp[s].np == 0) continue;
    if (f32)
      hipLaunchKernelGGL((k_diag_atomic<float, true, double>), dim3(nblocks(sp[s].np, kBlock)), dim3(kBlock), 0, st,
                         g, (int)sp[s].np, (const float*)sp[s].pos[0], (const float*)sp[s].pos[1],
                         (const float*)sp[s].pos[2], sp[s].cell, (const float*)sp[s].vel[0],
                         (const float*)sp[s].vel[1], (const float*)sp[s].vel[2], (const float*)sp[s].q,
                         (float)sp[s].q_const, a, a + nn, a + 4 * nn);
    else
      hipLaunchKernelGGL((k_diag_atomic<double, false, double>), dim3(nblocks(sp[s].np, kBlock)), dim3(kBlock), 0,
                         st, g, (int)sp[s].np, (const double*)sp[s].pos[0], (const double*)sp[s].pos[1],
                         (const double*)sp[s].pos[2], (const int32_t*)nullptr, (const double*)sp[s].vel[0],
                         (const double*)sp[s].vel[1], (const double*)sp[s].vel[2], (const double*)sp[s].q,
                         sp[s].q_const, (double*)rho, (double*)Jd, (double*)P);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (f32) {
    const unsigned blocks = (unsigned)std::min<int64_t>(nblocks(nn, kBlock), 4096);
    hipLaunchKernelGGL(k_add_rounded, dim3(blocks), dim3(kBlock), 0, st, nn, a, (float*)rho);
    hipLaunchKernelGGL(k_add_rounded, dim3(blocks), dim3(kBlock), 0, st, 3 * nn, a + nn, (float*)Jd);
    hipLaunchKernelGGL(k_add_rounded, dim3(blocks), dim3(kBlock), 0, st, 6 * nn, a + 4 * nn, (float*)P);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_deposit_atomic(const Grid& g, bool f32, const SpeciesArgs* sp, int ns, const void* B, void* J,
                                 void* M, hipStream_t st) {
  for (int s = 0; s < ns; ++s) {
    if (sp[s].np == 0) continue;
    const double beta = sp[s].qom * g.dt / 2.0;
    if (f32) {
      hipLaunchKernelGGL((k_deposit_atomic<float, true>), dim3(nblocks(sp[s].np, kBlock)), dim3(kBlock), 0, st, g,
                         sp[s].np, (const float*)sp[s].pos[0], (const float*)sp[s].pos[1],
                         (const float*)sp[s].pos[2], sp[s].cell, (const float*)sp[s].vel[0],
                         (const float*)sp[s].vel[1], (const float*)sp[s].vel[2], (const float*)sp[s].q,
                         (float)sp[s].q_const, (float)beta, (const float*)B, (float*)J, (float*)M);
    } else {
      hipLaunchKernelGGL((k_deposit_atomic<double, false>), dim3(nblocks(sp[s].np, kBlock)), dim3(kBlock), 0, st,
                         g, sp[s].np, (const double*)sp[s].pos[0], (const double*)sp[s].pos[1],
                         (const double*)sp[s].pos[2], (const int32_t*)nullptr, (const double*)sp[s].vel[0],
                         (const double*)sp[s].vel[1], (const double*)sp[s].vel[2], (const double*)sp[s].q,
                         sp[s].q_const, beta, (const double*)B, (double*)J, (double*)M);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t sort_workspace_bytes(const Grid& g, int64_t np) {
  int64_t nc = g.nn;
  int64_t ntiles = (nc + kScanTile - 1) / kScanTile;
  return align256(sizeof(int) * (size_t)np) * 2 + align256(sizeof(int) * (size_t)nc) +
         align256(sizeof(int) * (size_t)scan_sums_ints(nc));
}

// Scratch of the scan: one sum per tile at each level above the first (a
// level's sums are scanned, recursively, into the space after them).
int64_t scan_sums_ints(int64_t n) {
  int64_t total = 2;
  for (int64_t m = (n + kScanTile - 1) / kScanTile; ; m = (m + kScanTile - 1) / kScanTile) {
    total += 2 * (m + 1);
    if (m <= kScanTile) break;
  }
  return total;
}

hipError_t launch_exclusive_scan(const int* in, int64_t n, int* out, int* sums, hipStream_t st) {
  if (n < 0 || n >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if (ntiles <= kScanTile) {
    const unsigned nb = (unsigned)(ntiles > 0 ? ntiles : 1);
    hipLaunchKernelGGL(k_scan_tiles, dim3(nb), dim3(kScanBlock), 0, st, in, (int)n, out, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, sums, (int)ntiles, out + n);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanBlock), 0, st, out, (int)n, (const int*)sums,
                       (const int*)nullptr);
    return hipGetLastError();
  }
  // more tiles than one block scans: the tile sums are scanned recursively
  // into scan (ntiles + 1 values, the last one the total)
  int* scan = sums + ntiles + 1;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanBlock), 0, st, in, (int)n, out, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_exclusive_scan(sums, ntiles, scan, scan + ntiles + 1, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)ntiles), dim3(kScanBlock), 0, st, out, (int)n, (const int*)scan,
                     (const int*)(scan + ntiles));
  return hipGetLastError();
}

hipError_t launch_sort(const Grid& g, bool f32, const SpeciesArgs& src, const SpeciesArgs& dst,
                       int32_t* cell_start, int32_t* perm, void* ws, hipStream_t st) {
  const int64_t nc = g.nn;
  const int np = src.np;
  char* w = (char*)ws;
  int* keys = (int*)w;
  w += align256(sizeof(int) * (size_t)np);
  int* ranks = (int*)w;
  w += align256(sizeof(int) * (size_t)np);
  int* counts = (int*)w;
  w += align256(sizeof(int) * (size_t)nc);
  int* sums = (int*)w;
  const int ntiles = (int)((nc + kScanTile - 1) / kScanTile);
  hipError_t e = launch_zero(counts, sizeof(int) * (size_t)nc, st);   // a fill kernel: safe to capture
  if (e != hipSuccess) return e;
  if (np > 0) {
    if (f32)
      hipLaunchKernelGGL((k_sort_count<float, true>), dim3(nblocks(np, kBlock)), dim3(kBlock), 0, st, g, np,
                         (const float*)src.pos[0], (const float*)src.pos[1], (const float*)src.pos[2], src.cell,
                         counts, keys, ranks);
    else
      hipLaunchKernelGGL((k_sort_count<double, false>), dim3(nblocks(np, kBlock)), dim3(kBlock), 0, st, g, np,
                         (const double*)src.pos[0], (const double*)src.pos[1], (const double*)src.pos[2],
                         (const int32_t*)nullptr, counts, keys, ranks);
  }
  (void)ntiles;
  e = launch_exclusive_scan(counts, nc, cell_start, sums, st);
  if (e != hipSuccess) return e;
  if (np > 0) {
    if (f32)
      hipLaunchKernelGGL((k_sort_scatter<float, true>), dim3(nblocks(np, kBlock)), dim3(kBlock), 0, st, np, keys,
                         ranks, cell_start, (const float*)src.pos[0], (const float*)src.pos[1],
                         (const float*)src.pos[2], src.cell, (const float*)src.vel[0], (const float*)src.vel[1],
                         (const float*)src.vel[2], (const float*)src.q, (float*)dst.pos[0], (float*)dst.pos[1],
                         (float*)dst.pos[2], dst.cell, (float*)dst.vel[0], (float*)dst.vel[1],
                         (float*)dst.vel[2], (float*)const_cast<void*>(dst.q), perm);
    else
      hipLaunchKernelGGL((k_sort_scatter<double, false>), dim3(nblocks(np, kBlock)), dim3(kBlock), 0, st, np, keys,
                         ranks, cell_start, (const double*)src.pos[0], (const double*)src.pos[1],
                         (const double*)src.pos[2], (const int32_t*)nullptr, (const double*)src.vel[0],
                         (const double*)src.vel[1], (const double*)src.vel[2], (const double*)src.q,
                         (double*)dst.pos[0], (double*)dst.pos[1], (double*)dst.pos[2], (int32_t*)nullptr,
                         (double*)dst.vel[0], (double*)dst.vel[1], (double*)dst.vel[2],
                         (double*)const_cast<void*>(dst.q), perm);
  }
  return hipGetLastError();
}

}  // namespace ecsim
