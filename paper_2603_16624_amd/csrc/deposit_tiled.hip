// Tiled, LDS-binned moment deposit (Eqs. 1 and 3) over cell-sorted particles.
//
// Per cell the deposit is a small dense contraction. For corner pair (a, b)
// the weight product W_a W_b depends only on the class c = a + b in {0,1,2}^3
// (per dimension (1-xi)^2, xi (1-xi) or xi^2), so over the particles p of a
// cell
//   S[c][i] = sum_p v_i(p) m_c(p),   v = ((q beta / V) alpha_p (9 values),
//                                         (q / V) alpha_p v_p (3 values)),
// a (12 x K) by (K x 27) product. The stored block of every pair {a, b}
// receives S[a+b][0..8]; by the partition of unity sum_b W_b = 1 the current
// at corner a is J_a = sum_b S[a+b][9..11].
//
// Structure. A workgroup owns a brick of TX x TY x TZ cells. Each wavefront
// takes two cells at a time:
//   1. particle lanes (lanes 0-31: cell A, 32-63: cell B) recompute the
//      weights and alpha_p exactly as the mover does and write one record per
//      particle to LDS: the 12 values and the 9 per-dimension weight factors;
//   2. the contraction runs on the matrix cores: v_mfma 16x16x4 with rows =
//      the 12 values (padded to 16), columns = the 27 classes (two tiles of 16)
//      and K = 4 particles per instruction; FP32 sums are formed in blocks of
//      32 particles and the blocks combined with Kahan compensation;
//   3. the per-cell sums go to LDS (one writer per entry, no atomics);
// then, after a workgroup barrier, every (node, entry) of the brick gathers
// its <= 8 cell contributions and is added to the global J and M once.
#include "internal.h"

namespace ecsim {

namespace {

constexpr int kMaxTiledSpecies = 4;
constexpr int SCS = 268;        // per-cell sums: [27][9] mass-matrix classes, [8][3] corner currents, pad

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
  typedef f32x4 acc;
  __device__ __forceinline__ static acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of the 16x16 result held in register r of lane l (column l % 16)
  __device__ __forceinline__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct Mfma<double> {
  typedef f64x4 acc;
  __device__ __forceinline__ static acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int l, int r) { return (l >> 4) + 4 * r; }
};

template <typename T>
struct TSpecies {
  const T* pos[3];
  const T* vel[3];
  const T* q;
  T q_const;
  T beta;
  T beta_V;      // beta / V
  T inv_V;       // 1 / V
  const int32_t* cell_start;
};

template <typename T>
struct TArgs {
  TSpecies<T> s[kMaxTiledSpecies];
  int ns;
};

// Kahan compensated summation: the true running sum is s - c.
template <typename T>
__device__ __forceinline__ void kahan(T& s, T& c, T x) {
  T y = x - c;
  T t = s + y;
  c = (t - s) - y;
  s = t;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
struct PData {       // one particle's inputs, loaded ahead of use
  T x0, x1, x2, v0, v1, v2, q;
  int s;
  bool ok;
};

template <typename T>
__device__ __forceinline__ PData<T> load_particle(const TArgs<T>& args, const int* cnt, const int* beg, int total,
                                                  int ip) {
  PData<T> d{};
  d.ok = ip < total;
  if (d.ok) {
    int s = 0, idx = ip;
#pragma unroll
    for (int k = 0; k < kMaxTiledSpecies - 1; ++k)
      if (s == k && idx >= cnt[k]) { idx -= cnt[k]; s = k + 1; }
    const TSpecies<T>& sp = args.s[s];
    const int p = beg[s] + idx;
    d.s = s;
    d.x0 = sp.pos[0][p];
    d.x1 = sp.pos[1][p];
    d.x2 = sp.pos[2][p];
    d.v0 = sp.vel[0][p];
    d.v1 = sp.vel[1][p];
    d.v2 = sp.vel[2][p];
    d.q = sp.q ? sp.q[p] : sp.q_const;
  }
  return d;
}

// stored block k: offset o_k (same order as the C ABI)
__host__ __device__ constexpr int koff(int k, int d) {
  return k == 0 ? 0
       : k == 1 ? (d == 0 ? 1 : 0)
       : k < 5  ? (d == 0 ? k - 3 : d == 1 ? 1 : 0)
                : (d == 0 ? (k - 5) % 3 - 1 : d == 1 ? (k - 5) / 3 - 1 : 1);
}
// corner a of a cell pairs with a + o_k inside the cell: class 2a + o_k, else -1
__host__ __device__ constexpr int pair_class(int k, int a) {
  return ((a & 1) + koff(k, 0) < 0 || (a & 1) + koff(k, 0) > 1 || ((a >> 1) & 1) + koff(k, 1) < 0 ||
          ((a >> 1) & 1) + koff(k, 1) > 1 || ((a >> 2) & 1) + koff(k, 2) < 0 || ((a >> 2) & 1) + koff(k, 2) > 1)
             ? -1
             : (2 * (a & 1) + koff(k, 0)) + 3 * (2 * ((a >> 1) & 1) + koff(k, 1)) + 9 * (2 * ((a >> 2) & 1) + koff(k, 2));
}

// Records in LDS are stored transposed, rec[row][slot] with a row stride of
// 66 slots (64 particles + 2): the MFMA operand reads of 16 lanes with
// consecutive rows and 2 lane groups then hit 32 different banks.
constexpr int kSlots = 66;
constexpr int kRows = 44;       // 12 values, 27 class weights, 5 spare rows
constexpr int kRowB = 39;       // spare row: corner magnetic field of the two cells
constexpr int kRowT = 40;       // spare rows 40..42: current class sums of the two cells

template <typename T, int TX, int TY, int TZ, int NW>
__global__ void __launch_bounds__(NW * 64) k_deposit_tiled(Grid g, TArgs<T> args, int ntx, int nty, int ntz,
                                                          const T* __restrict__ B, T* __restrict__ J,
                                                          T* __restrict__ M) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc;
  constexpr int NX = TX + 1, NY = TY + 1, NZ = TZ + 1, NN = NX * NY * NZ;
  constexpr int NCELL = TX * TY * TZ;
  constexpr int NPAIR = (NCELL + 1) / 2;
  constexpr int WREC = kRows * kSlots;
  // one LDS block: the wavefront records first (so that their offsets fit the
  // 16-bit immediate of ds_read), then the per-cell sums
  __shared__ __attribute__((aligned(16))) T smem[NW * WREC + NCELL * SCS];
  T* const scell = smem + NW * WREC;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int half = lane >> 5;
  const int hl = lane & 31;
  const int col = lane & 15;                    // MFMA column (class) of this lane
  const int grp = lane >> 4;                    // MFMA k-group of this lane

  // tile coordinates; blocks are spread so that each XCD gets contiguous tiles
  const int ntiles = ntx * nty * ntz;
  int b = blockIdx.x;
  {
    constexpr int nxcd = 8;
    const int per = ntiles / nxcd;
    if (per * nxcd == ntiles) b = (b % nxcd) * per + b / nxcd;
  }
  const int tx = b % ntx, ty = (b / ntx) % nty, tz = b / (ntx * nty);
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;

  for (int i = tid; i < NCELL * SCS; i += NW * 64) scell[i] = T(0);
  for (int i = tid; i < NW * WREC; i += NW * 64) smem[i] = T(0);
  __syncthreads();

  T* const wrec = smem + wave * WREC;
  // this lane's MFMA operand base: row col, slot grp (cell A) / 32 + grp (cell B)
  const T* const opnd = wrec + col * kSlots + grp;

  for (int pair = wave; pair < NPAIR; pair += NW) {
    // my half's cell
    const int lc = 2 * pair + half;
    const int lx = lc % TX, ly = (lc / TX) % TY, lz = lc / (TX * TY);
    const int cx = x0 + lx, cy = y0 + ly, cz = z0 + lz;
    const bool valid = (lc < NCELL) && cx < g.nx && cy < g.ny && cz < g.nz;
    const int64_t cell = valid ? cx + (int64_t)g.nx * (cy + (int64_t)g.ny * cz) : 0;
    int cnt[kMaxTiledSpecies];
    int beg[kMaxTiledSpecies];
    int total = 0;
#pragma unroll
    for (int s = 0; s < kMaxTiledSpecies; ++s) {
      cnt[s] = 0;
      beg[s] = 0;
      if (s < args.ns && valid) {
        beg[s] = args.s[s].cell_start[cell];
        cnt[s] = args.s[s].cell_start[cell + 1] - beg[s];
      }
      total += cnt[s];
    }
    const int cntA = __builtin_amdgcn_readfirstlane(__shfl(total, 0));
    const int cntB = __builtin_amdgcn_readfirstlane(__shfl(total, 32));
    const int cmax = cntA > cntB ? cntA : cntB;
    // corner nodes of the cell; lanes 0..23 of each half fetch the magnetic field
    Stencil<T> st{};
    st.i[0] = valid ? cx : 0;
    st.i[1] = valid ? cy : 0;
    st.i[2] = valid ? cz : 0;
    st.ip[0] = wrap_up(st.i[0], g.nx);
    st.ip[1] = wrap_up(st.i[1], g.ny);
    st.ip[2] = wrap_up(st.i[2], g.nz);
    T* const myB = wrec + kRowB * kSlots + 24 * half;
    if (hl < 24) myB[hl] = B[(hl >> 3) * g.nn + corner_node(g, st, hl & 7)];
    PData<T> pd = load_particle(args, cnt, beg, total, hl);
    wave_sync();
    T Bn[3][8];
#pragma unroll
    for (int i = 0; i < 24; ++i) Bn[i >> 3][i & 7] = myB[i];

    // running sums of the two cells: [cell][tile][reg]
    T S[2][2][4], C[2][2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) { S[h][t][r] = T(0); C[h][t][r] = T(0); }

    for (int ch = 0; ch < cmax; ch += 32) {
      // ---- 1. particle lanes: one record column per lane ----
      T r[39];
#pragma unroll
      for (int i = 0; i < 39; ++i) r[i] = T(0);
      if (pd.ok) {
        const TSpecies<T>& sp = args.s[pd.s];
        Stencil<T> ps = st;
        if constexpr (sizeof(T) == 4) {
          ps.w1[0] = pd.x0; ps.w1[1] = pd.x1; ps.w1[2] = pd.x2;
          ps.w0[0] = T(1) - pd.x0; ps.w0[1] = T(1) - pd.x1; ps.w0[2] = T(1) - pd.x2;
        } else {
          // the cell of a sorted particle is its range's cell
          Stencil<double> s2 = stencil_abs(g, pd.x0, pd.x1, pd.x2);
#pragma unroll
          for (int d = 0; d < 3; ++d) { ps.w0[d] = s2.w0[d]; ps.w1[d] = s2.w1[d]; }
        }
        T W[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) W[a] = corner_weight(ps, a);
        Vec3<T> Bp{T(0), T(0), T(0)};
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          Bp.x = fma(W[a], Bn[0][a], Bp.x);
          Bp.y = fma(W[a], Bn[1][a], Bp.y);
          Bp.z = fma(W[a], Bn[2][a], Bp.z);
        }
        T al[9];
        rotation(Bp, sp.beta, al);
        Vec3<T> vh = matvec(al, Vec3<T>{pd.v0, pd.v1, pd.v2});
        const T cm = pd.q * sp.beta_V;
        const T cj = pd.q * sp.inv_V;
#pragma unroll
        for (int i = 0; i < 9; ++i) r[i] = cm * al[i];
        r[9] = cj * vh.x;
        r[10] = cj * vh.y;
        r[11] = cj * vh.z;
        T f[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          f[d][0] = ps.w0[d] * ps.w0[d];
          f[d][1] = ps.w0[d] * ps.w1[d];
          f[d][2] = ps.w1[d] * ps.w1[d];
        }
#pragma unroll
        for (int c = 0; c < 27; ++c) r[12 + c] = (f[0][c % 3] * f[1][(c / 3) % 3]) * f[2][c / 9];
      }
#pragma unroll
      for (int i = 0; i < 39; ++i) wrec[i * kSlots + lane] = r[i];
      wave_sync();
      // prefetch the next block's particles while this block is reduced
      if (ch + 32 < cmax) pd = load_particle(args, cnt, beg, total, ch + 32 + hl);

      // ---- 2. matrix cores: S[value][class] += sum over 4 particles per step ----
      // records past a cell's count are zero, so all 8 steps of a block run
      acc_t dA0 = {0, 0, 0, 0}, dA1 = {0, 0, 0, 0}, dB0 = {0, 0, 0, 0}, dB1 = {0, 0, 0, 0};
#pragma unroll
      for (int k4 = 0; k4 < 32; k4 += 4) {
        const T aA = opnd[k4];
        const T aB = opnd[32 + k4];
        const T bA0 = opnd[12 * kSlots + k4];
        const T bB0 = opnd[12 * kSlots + 32 + k4];
        const T bA1 = opnd[28 * kSlots + k4];
        const T bB1 = opnd[28 * kSlots + 32 + k4];
        dA0 = MF::run(aA, bA0, dA0);
        dB0 = MF::run(aB, bB0, dB0);
        dA1 = MF::run(aA, bA1, dA1);
        dB1 = MF::run(aB, bB1, dB1);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if constexpr (sizeof(T) == 4) {
          kahan(S[0][0][q], C[0][0][q], dA0[q]);
          kahan(S[0][1][q], C[0][1][q], dA1[q]);
          kahan(S[1][0][q], C[1][0][q], dB0[q]);
          kahan(S[1][1][q], C[1][1][q], dB1[q]);
        } else {
          S[0][0][q] += dA0[q];
          S[0][1][q] += dA1[q];
          S[1][0][q] += dB0[q];
          S[1][1][q] += dB1[q];
        }
      }
      wave_sync();
    }

    // ---- 3. per-cell sums to LDS: mass-matrix classes, current classes ----
    T* const tcur = wrec + kRowT * kSlots;     // [2][84]
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int lch = 2 * pair + h;
      if (lch >= NCELL) continue;
      T* sc = scell + lch * SCS;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int cls = t * 16 + col;
        if (cls >= 27) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = MF::row(lane, q);
          T v = S[h][t][q];
          if constexpr (sizeof(T) == 4) v -= C[h][t][q];
          if (row < 9) sc[cls * 9 + row] = v;
          else if (row < 12) tcur[h * 84 + cls * 3 + (row - 9)] = v;
        }
      }
    }
    wave_sync();
    // corner currents J_a = sum_b T_{a+b}: lanes 0..23 of each half
    if (hl < 24 && lc < NCELL) {
      const int a = hl / 3, comp = hl % 3;
      const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      const T* tc = tcur + half * 84;
      T s = T(0);
#pragma unroll
      for (int bb = 0; bb < 8; ++bb) {
        const int cls = (ax + (bb & 1)) + 3 * (ay + ((bb >> 1) & 1)) + 9 * (az + ((bb >> 2) & 1));
        s += tc[cls * 3 + comp];
      }
      scell[lc * SCS + 243 + 3 * a + comp] = s;
    }
    wave_sync();
  }
  __syncthreads();

  // ---- gather every (entry, node) of the brick and add it to J and M ----
  // items: (ij, node) for the mass matrix, then (component, node) for J
  constexpr int NITEM = 9 * NN + 3 * NN;
  for (int it = tid; it < NITEM; it += NW * 64) {
    const bool is_m = it < 9 * NN;
    const int ln = is_m ? it % NN : (it - 9 * NN) % NN;
    const int sub = is_m ? it / NN : (it - 9 * NN) / NN;   // ij, or the current component
    const int nx_ = ln % NX, ny_ = (ln / NX) % NY, nz_ = ln / (NX * NY);
    // cells n - a that exist in this brick
    int vmask = 0;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int lcx = nx_ - (a & 1), lcy = ny_ - ((a >> 1) & 1), lcz = nz_ - ((a >> 2) & 1);
      if (lcx >= 0 && lcx < TX && lcy >= 0 && lcy < TY && lcz >= 0 && lcz < TZ) vmask |= 1 << a;
    }
    const int cbase = nx_ + TX * (ny_ + TY * nz_);          // cell index of n (may lie outside)
    const int gx = (x0 + nx_) % g.nx, gy = (y0 + ny_) % g.ny, gz = (z0 + nz_) % g.nz;
    const int64_t gn = gx + (int64_t)g.nx * (gy + (int64_t)g.ny * gz);
    if (is_m) {
#pragma unroll
      for (int k = 0; k < 14; ++k) {
        T v = T(0);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const int cls = pair_class(k, a);
          if (cls < 0) continue;
          if (vmask & (1 << a)) {
            const int cidx = cbase - ((a & 1) + TX * (((a >> 1) & 1) + TY * ((a >> 2) & 1)));
            v += scell[cidx * SCS + cls * 9 + sub];
          }
        }
        if (v != T(0)) unsafeAtomicAdd(M + (int64_t)(k * 9 + sub) * g.nn + gn, v);
      }
    } else {
      T v = T(0);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        if (vmask & (1 << a)) {
          const int cidx = cbase - ((a & 1) + TX * (((a >> 1) & 1) + TY * ((a >> 2) & 1)));
          v += scell[cidx * SCS + 243 + 3 * a + sub];
        }
      }
      if (v != T(0)) unsafeAtomicAdd(J + (int64_t)sub * g.nn + gn, v);
    }
  }
}

template <typename T, int TX, int TY, int TZ, int NW>
hipError_t launch_T(const Grid& g, const SpeciesArgs* sp, int ns, const void* B, void* J, void* M, hipStream_t st) {
  TArgs<T> a{};
  a.ns = ns;
  for (int s = 0; s < ns; ++s) {
    for (int d = 0; d < 3; ++d) {
      a.s[s].pos[d] = (const T*)sp[s].pos[d];
      a.s[s].vel[d] = (const T*)sp[s].vel[d];
    }
    a.s[s].q = (const T*)sp[s].q;
    a.s[s].q_const = (T)sp[s].q_const;
    a.s[s].beta = (T)(sp[s].qom * g.dt / 2.0);
    a.s[s].beta_V = (T)(sp[s].qom * g.dt / 2.0 / g.V);
    a.s[s].inv_V = (T)(1.0 / g.V);
    a.s[s].cell_start = sp[s].cell_start;
  }
  const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + TZ - 1) / TZ;
  const int ntiles = ntx * nty * ntz;
  hipLaunchKernelGGL((k_deposit_tiled<T, TX, TY, TZ, NW>), dim3(ntiles), dim3(NW * 64), 0, st, g, a, ntx, nty, ntz,
                     (const T*)B, (T*)J, (T*)M);
  return hipGetLastError();
}

}  // namespace

bool tiled_supported(const Grid& g) { return g.nn > 0; }

hipError_t launch_deposit_tiled(const Grid& g, bool f32, const SpeciesArgs* sp, int ns, const void* B, void* J,
                                void* M, hipStream_t st) {
  if (ns > kMaxTiledSpecies) return launch_deposit_atomic(g, f32, sp, ns, B, J, M, st);
  if (f32) return launch_T<float, 4, 4, 4, 8>(g, sp, ns, B, J, M, st);
  return launch_T<double, 4, 4, 2, 4>(g, sp, ns, B, J, M, st);
}

}  // namespace ecsim
