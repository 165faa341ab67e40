// Tiled moment deposit (Eqs. 1 and 3) over cell-grouped particles, and the
// grouped mover (Eqs. 4, 5, 8) that feeds it.
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
// Particles are grouped by per-species cell ranges (cell_start) that may be
// stale. One pass, per brick of cells, runs over the ranges first: the
// grouped mover moves every particle with the corner fields of its range's
// cell staged in LDS (a particle already outside that cell is left to a small
// kernel that reads its fields from memory), or, for a deposit alone, the
// ranges are only checked. Every particle that is not in its range's cell
// afterwards goes to a stray list, which is counting-sorted by cell.
//
// The deposit kernel: a workgroup owns a brick of TX x TY x TZ cells; each
// cell's particles are its species ranges (entries outside the cell carry
// zero charge) followed by its entries of the sorted stray list. Each
// wavefront takes cells wave, wave + NW, ... of the brick, one at a time, in
// blocks of 64 of the cell's particles:
//   1. each lane takes one particle and writes a record to LDS: the 12 values
//      and the 27 class weights, with the mover's stencil and field gather
//      (alpha_p bit for bit in FP64, to rounding in FP32);
//   2. the contraction runs on the matrix cores: v_mfma 16x16x4 with rows =
//      the 12 values (padded to 16), columns = the 27 classes (two tiles of 16)
//      and K = 4 particles per instruction; FP32 sums are formed in blocks of
//      64 particles and the blocks combined with Kahan compensation;
//   3. a finished cell's sums (27 x 9 mass-matrix classes and 8 x 3 corner
//      currents) go to its record in HBM, written once, no atomics.
// The flush kernel then stages bricks of cell records in LDS and gives every
// (node, entry) of J and M the sum of its <= 8 cell contributions, written
// (or added, when moments accumulate over several calls) once.
#include "internal.h"

namespace ecsim {

namespace {

constexpr int kMaxTiledSpecies = 4;
constexpr int kStraySlot = kMaxTiledSpecies;  // range slot of the sorted stray list
constexpr int kSlots5 = kMaxTiledSpecies + 1;
constexpr int kItemShift = 28;              // stray item = species << 28 | particle index
constexpr int kUnmoved = 1 << 30;           // flag: listed before its move
constexpr int kIndexMask = (1 << kItemShift) - 1;
constexpr int SCS = 268;                    // per-cell sums: [27][9] mass-matrix classes, [8][3] currents, pad

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
  T* pos[3];
  T* vel[3];
  int32_t* cell;
  const T* q;
  T q_const;
  T beta;
  T beta_V;      // beta / V
  T inv_V;       // 1 / V
  double inv_qom;
  const int32_t* cell_start;
  int np;
};

// The strays' state copied out of the species arrays in cell order (the
// deposit reads it without indirection); sp holds each stray's species.
template <typename T>
struct StrayData {
  T* pos[3];
  T* vel[3];
  T* q;
  int32_t* cell;
  int32_t* sp;
};

// Where the regrouping deposit writes a species' particles in cell order, and
// the cell ranges (start[c] .. start[c + 1]) it writes them in.
template <typename T>
struct RegroupDst {
  T* pos[3];
  T* vel[3];
  T* q;              // NULL for a constant-charge species
  int32_t* cell;     // FP32 form only
  int32_t* start;
  int np;
};

template <typename T>
struct TArgs {
  TSpecies<T> s[kMaxTiledSpecies];
  int ns;
  const T* Bdep;       // magnetic field of the deposit
  const T* Emove;      // mover fields
  const T* Bmove;
  T dth[3];            // dt / h
  int* stray_count;
  int* stray_item;
  int* stray_cell;
  StrayData<T> ul;        // the listed strays' state, in list order
  const int* ind_start;   // the stray list sorted by cell: ranges
  StrayData<T> sd;        // ... and the strays' state in that order
  const void* zero;       // 64 zero bytes: the load target of idle lanes
  void* sink;             // the store target of idle lanes (never read)
  double* ke;
  // regrouping (NULL stay: off): per (species, cell) the particles that stayed
  // in their range's cell and the listed strays, and the targets
  int* stay;
  int* scount;
  RegroupDst<T> dst[kMaxTiledSpecies];
  T* csum;   // per-cell sums [cells][SCS], written by the deposit, read by the node flush
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

// A particle's state as the mover writes it back: position (FP32: in-cell
// offsets), velocity, charge and cell.
template <typename T>
struct SRec {
  T x0, x1, x2, v0, v1, v2, q;
  int c;
};

// A wavefront's strays (item, cell and state) collect in LDS and go to the
// list in list order when the buffer is full (one returning atomic per
// kWaveList entries) and at the end (one atomic per workgroup). 96 entries
// (and a 5 KB map below) keep the FP32 mover's workgroup within 32 KB of
// LDS: 5 waves per SIMD instead of 4 (457 -> 441 us at 64^3).
constexpr int kWaveList = 96;

template <typename T>
struct WaveBuf {
  int item[kWaveList];
  int cell[kWaveList];
  T val[7][kWaveList];   // pos[3], vel[3], q
  int vcell[kWaveList];
};

template <typename T>
struct WaveStrays {
  int fill = 0;   // wavefront-uniform

  // copies the buffer's first fill entries to the list at base
  template <typename TA>
  __device__ __forceinline__ void copy_out(const TA& args, const WaveBuf<T>& b, int lane, int base) const {
    const StrayData<T>& u = args.ul;
    for (int i = lane; i < fill; i += 64) {
      const int o = base + i;
      args.stray_item[o] = b.item[i];
      args.stray_cell[o] = b.cell[i];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        u.pos[k][o] = b.val[k][i];
        u.vel[k][o] = b.val[3 + k][i];
      }
      u.q[o] = b.val[6][i];
      u.cell[o] = b.vcell[i];
    }
  }

  // lists the lanes with stray set (reached by the whole wavefront)
  template <typename TA>
  __device__ __forceinline__ void put(const TA& args, WaveBuf<T>& b, int lane, bool stray, int item, int cell,
                                      const SRec<T>& r) {
    const unsigned long long bal = __ballot(stray);
    const int nst = __popcll(bal);
    if (nst == 0) return;
    if (fill + nst > kWaveList) {   // full: to the list
      int rv = 0;
      if (lane == 0) rv = atomicAdd(args.stray_count, fill);
      wave_sync();
      copy_out(args, b, lane, __builtin_amdgcn_readfirstlane(rv));
      wave_sync();
      fill = 0;
    }
    if (stray) {
      const int i = fill + __popcll(bal & ((1ull << lane) - 1ull));
      b.item[i] = item;
      b.cell[i] = cell;
      b.val[0][i] = r.x0;
      b.val[1][i] = r.x1;
      b.val[2][i] = r.x2;
      b.val[3][i] = r.v0;
      b.val[4][i] = r.v1;
      b.val[5][i] = r.v2;
      b.val[6][i] = r.q;
      b.vcell[i] = r.c;
    }
    fill += nst;
  }
};

// Particle arrays are addressed through pointers held in LDS; these casts
// give the compiler the global address space (global_load/store, not flat).
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

template <typename T>
struct PData {       // one particle's inputs, loaded ahead of use
  T x0, x1, x2, v0, v1, v2, q;
  int c;             // stored cell (FP32 form)
  int s, p;
  bool ok;
};

template <typename T>
__device__ __forceinline__ Stencil<T> particle_stencil(const Grid& g, T x0, T x1, T x2, int c);
template <>
__device__ __forceinline__ Stencil<float> particle_stencil<float>(const Grid& g, float x0, float x1, float x2, int c) {
  return stencil_cell(g, c, x0, x1, x2);
}
template <>
__device__ __forceinline__ Stencil<double> particle_stencil<double>(const Grid& g, double x0, double x1, double x2,
                                                                   int) {
  return stencil_abs(g, x0, x1, x2);
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

// Where a deposit lane reads its particle: slots 0..3 the species arrays,
// kStraySlot the sorted strays, kZeroSlot a zero block (idle lanes). Every
// pointer is valid, so the loads need no branch.
constexpr int kZeroSlot = kStraySlot + 1;
constexpr int kMapCap = 5120;   // grouped pass: largest brick list with a position -> range map
template <typename T>
struct PtrSet {
  const T* pos[3];
  const T* vel[3];
  const T* q;
  const int32_t* cell;
  const int32_t* sp;
  T qconst;   // added to the loaded q: the charge of a constant-charge species
  // index masks: all ones for a per-particle array, 0 for the zero block
  int qmask, cmask, smask;
};

template <typename T>
__device__ __forceinline__ PtrSet<T> ptr_set_species(const TSpecies<T>& sp, const void* zero) {
  PtrSet<T> P;
  for (int d = 0; d < 3; ++d) {
    P.pos[d] = sp.pos[d];
    P.vel[d] = sp.vel[d];
  }
  P.q = sp.q ? sp.q : (const T*)zero;
  P.qconst = sp.q ? T(0) : sp.q_const;
  P.cell = sp.cell ? sp.cell : (const int32_t*)zero;
  P.sp = (const int32_t*)zero;
  P.qmask = sp.q ? -1 : 0;
  P.cmask = sp.cell ? -1 : 0;
  P.smask = 0;
  return P;
}

template <typename T>
__device__ __forceinline__ PtrSet<T> ptr_set_strays(const StrayData<T>& sd) {
  PtrSet<T> P;
  for (int d = 0; d < 3; ++d) {
    P.pos[d] = sd.pos[d];
    P.vel[d] = sd.vel[d];
  }
  P.q = sd.q;
  P.qconst = T(0);
  P.cell = sd.cell;
  P.sp = sd.sp;
  P.qmask = P.cmask = P.smask = -1;
  return P;
}

template <typename T>
__device__ __forceinline__ PtrSet<T> ptr_set_zero(const void* zero) {
  PtrSet<T> P;
  const T* z = (const T*)zero;
  for (int d = 0; d < 3; ++d) P.pos[d] = P.vel[d] = z;
  P.q = z;
  P.qconst = T(0);
  P.cell = P.sp = (const int32_t*)zero;
  P.qmask = P.cmask = P.smask = 0;
  return P;
}

// Fills the LDS tables of species and read slots (constant kernel-argument
// indices only, so nothing goes through private memory).
template <typename T>
__device__ __forceinline__ void fill_tables(const TArgs<T>& args, TSpecies<T>* lsp, PtrSet<T>* lptr, int tid) {
#pragma unroll
  for (int k = 0; k < kMaxTiledSpecies; ++k) {
    if (tid == k) {
      const TSpecies<T>& sp = k < args.ns ? args.s[k] : args.s[0];
      lsp[k] = sp;
      if (lptr) lptr[k] = ptr_set_species(sp, args.zero);
    }
  }
  if (lptr && tid == kStraySlot) lptr[kStraySlot] = ptr_set_strays(args.sd);
  if (lptr && tid == kZeroSlot) lptr[kZeroSlot] = ptr_set_zero<T>(args.zero);
}

// Particle ip of a cell whose particles are the ranges cnt/beg of the species
// slots and then the stray slot, loaded without branches.
template <typename T>
using LdsPtrSet = const __attribute__((address_space(3))) PtrSet<T>;

// A cell's particle list is its slots' ranges back to back: list position ip
// lies in slot k when end[k-1] <= ip < end[k], at particle beg[k] + ip - end[k-1].
// With dlt[k] = beg[k] - end[k-1] stored as d0 = dlt[0] and the steps
// inc[k] = dlt[k+1] - dlt[k], the index is ip + d0 + the steps of the ends
// passed: sums of selects, which the compiler cannot turn into an indexed
// (private memory) table.
struct Ranges {
  int end[kSlots5 - 1], inc[kSlots5 - 1], d0, total;
};

__device__ __forceinline__ Ranges select_ranges(bool a, const Ranges& x, const Ranges& y) {
  Ranges r;
#pragma unroll
  for (int k = 0; k < kSlots5 - 1; ++k) {
    r.end[k] = a ? x.end[k] : y.end[k];
    r.inc[k] = a ? x.inc[k] : y.inc[k];
  }
  r.d0 = a ? x.d0 : y.d0;
  r.total = a ? x.total : y.total;
  return r;
}

template <typename T>
__device__ __forceinline__ PData<T> load_dep(LdsPtrSet<T>* lptr, const Ranges& r, int ip) {
  PData<T> d;
  d.ok = ip < r.total;
  // slot and particle index by compares against the slot ends (branch-free;
  // constant indices only, so no private memory)
  int slot = 0, dl = r.d0;
#pragma unroll
  for (int k = 0; k < kSlots5 - 1; ++k) {
    const bool past = ip >= r.end[k];
    slot += past ? 1 : 0;
    dl += past ? r.inc[k] : 0;
  }
  const int ts = d.ok ? slot : kZeroSlot;
  const int pi = d.ok ? ip + dl : 0;
  LdsPtrSet<T>& P = lptr[ts];   // LDS reads (a generic pointer would make them flat loads)
  // raw loads only: nothing here may use a loaded value, or the compiler
  // waits for the loads at once (see dep_species, dep_charge)
  d.x0 = gld(P.pos[0] + pi);
  d.x1 = gld(P.pos[1] + pi);
  d.x2 = gld(P.pos[2] + pi);
  d.v0 = gld(P.vel[0] + pi);
  d.v1 = gld(P.vel[1] + pi);
  d.v2 = gld(P.vel[2] + pi);
  d.q = gld(P.q + (pi & P.qmask));
  d.c = sizeof(T) == 4 ? gld(P.cell + (pi & P.cmask)) : 0;
  d.s = gld(P.sp + (pi & P.smask));   // the species of a stray
  d.p = ts;                           // the slot
  return d;
}

// species and charge of a loaded deposit particle
template <typename T>
__device__ __forceinline__ int dep_species(const PData<T>& d) {
  return d.p == kStraySlot ? d.s : (d.p < kMaxTiledSpecies ? d.p : 0);
}
template <typename T>
__device__ __forceinline__ T dep_charge(const PData<T>& d, LdsPtrSet<T>* lptr) {
  return d.q + lptr[d.p].qconst;
}

// A cell of a brick (local index lc).
struct BrickCell {
  int lc, cell, cx, cy, cz;
  bool valid;
};

template <int TX, int TY, int TZ>
__device__ __forceinline__ BrickCell brick_cell(const Grid& g, int x0, int y0, int z0, int lc) {
  BrickCell c;
  c.lc = lc;
  c.cx = x0 + lc % TX;
  c.cy = y0 + (lc / TX) % TY;
  c.cz = z0 + lc / (TX * TY);
  c.valid = lc < TX * TY * TZ && c.cx < g.nx && c.cy < g.ny && c.cz < g.nz;
  c.cell = c.valid ? c.cx + g.nx * (c.cy + g.ny * c.cz) : -1;
  return c;
}

// regrouping: where a cell's particles of each species start in the targets
struct DStart {
  int v[kMaxTiledSpecies];
};
template <typename T>
__device__ __forceinline__ DStart load_dstart(const TArgs<T>& args, const BrickCell& c) {
  DStart d;
  const int cl = c.valid ? c.cell : 0;
#pragma unroll
  for (int s = 0; s < kMaxTiledSpecies; ++s) d.v[s] = gld(args.dst[s < args.ns ? s : 0].start + cl);
  return d;
}

// cell range loads, issued one cell (pair) ahead of their use
struct RangeLd {
  int lo[kSlots5], hi[kSlots5];
};
template <typename T, int NSLOT>
__device__ __forceinline__ RangeLd load_ranges(const TArgs<T>& args, const TSpecies<T>* lsp, const BrickCell& c) {
  RangeLd r{};
  const int cl = c.valid ? c.cell : 0;
#pragma unroll
  for (int s = 0; s < kMaxTiledSpecies; ++s) {
    const int32_t* cs = lsp[s].cell_start;   // unused species alias species 0
    r.lo[s] = gld(cs + cl);                  // global loads (not flat: those would count as LDS too)
    r.hi[s] = gld(cs + cl + 1);
  }
  if constexpr (NSLOT > kStraySlot) {
    r.lo[kStraySlot] = gld(args.ind_start + cl);
    r.hi[kStraySlot] = gld(args.ind_start + cl + 1);
  }
  return r;
}

template <typename T, int NSLOT>
__device__ __forceinline__ Ranges make_ranges(const TArgs<T>& args, const RangeLd& r, const BrickCell& c) {
  static_assert(NSLOT == kSlots5, "ranges cover every slot");
  Ranges q;
  int e = 0, prev = 0;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const bool used = s == kStraySlot || s < args.ns;
    const int dlt = r.lo[s] - e;
    if (s == 0) q.d0 = dlt;
    else q.inc[s - 1] = dlt - prev;
    prev = dlt;
    e += (c.valid && used) ? r.hi[s] - r.lo[s] : 0;
    if (s < NSLOT - 1) q.end[s] = e;
  }
  q.total = e;
  return q;
}

constexpr int kRec = 24;   // record rows: 12 values, 3 + 9 weight factors

// A particle's record: the 12 values ((q beta / V) alpha, (q / V) alpha v)
// and the factors of its 27 class weights, from the deposit field B1 at its
// position: the x factors f_x[cx] (3) and the products f_y[cy] f_z[cz] (9,
// at cy + 3 cz); the weight of class cx + 3 (cy + 3 cz) is their product,
// formed where the matrix cores take it.
// FP64: alpha from rotation() (the mover's routine, so the two agree bit for
// bit). FP32: alpha = N / D with N = I + b b^T - [b x], b = beta B, written
// into the record with the charge factors folded into 1/D (one product per
// entry instead of two).
template <typename T>
__device__ __forceinline__ void particle_record(const Stencil<T>& ps, const Vec3<T>& B1, const Vec3<T>& v, T q,
                                                const TSpecies<T>& sp, T r[kRec]) {
  if constexpr (sizeof(T) == 4) {
    const T bx = sp.beta * B1.x, by = sp.beta * B1.y, bz = sp.beta * B1.z;
    const T xx = bx * bx, yy = by * by, zz = bz * bz, xy = bx * by, xz = bx * bz, yz = by * bz;
    const T inv = __builtin_amdgcn_rcpf(T(1) + ((xx + yy) + zz));
    const T n[9] = {T(1) + xx, xy + bz, xz - by, xy - bz, T(1) + yy, yz + bx, xz + by, yz - bx, T(1) + zz};
    const T cmi = (q * sp.beta_V) * inv;
    const T cji = (q * sp.inv_V) * inv;
#pragma unroll
    for (int i = 0; i < 9; ++i) r[i] = cmi * n[i];
    r[9] = cji * fma(n[2], v.z, fma(n[1], v.y, n[0] * v.x));
    r[10] = cji * fma(n[5], v.z, fma(n[4], v.y, n[3] * v.x));
    r[11] = cji * fma(n[8], v.z, fma(n[7], v.y, n[6] * v.x));
  } else {
    T al[9];
    rotation(B1, sp.beta, al);
    const Vec3<T> vh = matvec(al, v);
    const T cm = q * sp.beta_V;
    const T cj = q * sp.inv_V;
#pragma unroll
    for (int i = 0; i < 9; ++i) r[i] = cm * al[i];
    r[9] = cj * vh.x;
    r[10] = cj * vh.y;
    r[11] = cj * vh.z;
  }
  T f[3][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    f[d][0] = ps.w0[d] * ps.w0[d];
    f[d][1] = ps.w0[d] * ps.w1[d];
    f[d][2] = ps.w1[d] * ps.w1[d];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) r[12 + c] = f[0][c];
#pragma unroll
  for (int c = 0; c < 9; ++c) r[15 + c] = f[1][c % 3] * f[2][c / 3];
}

// Records in LDS are stored transposed, rec[row][slot] with a row stride of
// 66 slots (64 particles + 2): the matrix-core operand reads of 16 lanes with
// consecutive rows and 2 lane groups then hit 32 different banks. Rows 24-25
// hold the cell's current class sums at the end of a cell (read as operands
// only by the unused classes 27-30). A 4-wavefront workgroup needs 27 KB of
// LDS (FP32), so four workgroups fit a CU.
constexpr int kSlots = 66;
constexpr int kRows = 26;
constexpr int kTcur = kRec * kSlots;       // [27][3]: current class sums (end of a cell)


// ---------------------------------------------------------------------------
// grouped pass over the cell ranges: with MOVE the mover, else a check
// ---------------------------------------------------------------------------
// A workgroup owns a brick of TX x TY x TZ cells. It stages the mover fields
// E^{n+theta}, B^n on the brick's nodes plus a one-cell halo in LDS, then its
// wavefronts run through the brick's particles -- the species ranges of its
// cells, taken as one list -- 64 at a time, the next block's loads issued
// before the current block is computed. With MOVE a particle whose cell lies
// in the halo'd box is moved with the staged fields (the same gathers,
// rotation and push as everywhere else) and written back, and listed if it
// is now outside its range's cell; a particle beyond the box is listed
// unmoved (with its range's cell) for the stray mover. Without MOVE a
// particle outside its range's cell is listed with its cell.
template <typename T, int TX, int TY, int TZ, int NW, bool MOVE>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
k_group(Grid g, TArgs<T> args, int ntx, int nty, int ntz) {
  constexpr int NCELL = TX * TY * TZ;
  constexpr int HX = TX + 3, HY = TY + 3, HZ = TZ + 3, HN = HX * HY * HZ;   // halo'd node box
  constexpr int NR = NCELL * kMaxTiledSpecies;                            // ranges: cell-major
  constexpr int NT = NW * 64;
  static_assert(NR <= NT, "one range per thread");
  __shared__ T fld[MOVE ? 6 * HN : 1];
  __shared__ int rbeg[NR];
  __shared__ int roff[NR + 1];
  __shared__ int rleft[NR];   // regrouping: particles of each range listed as strays
  __shared__ int wsum[NW];
  __shared__ double red[NW];
  __shared__ TSpecies<T> lsp[kMaxTiledSpecies];
  __shared__ int wst[NW];
  __shared__ WaveBuf<T> slist[NW];
  __shared__ void* lsink;   // in LDS beside the species table: selects between them stay LDS reads
  // list position -> range, for bricks of at most kMapCap particles
  __shared__ uint8_t rmap[kMapCap];
  static_assert(NR <= 256, "range indices fit a byte");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  int x0, y0, z0;
  brick_origin<TX, TY, TZ>(ntx, nty, ntz, x0, y0, z0);
  fill_tables<T>(args, lsp, nullptr, tid);
  if (tid == 0) lsink = args.sink;
  // range r = (cell lc = r / 4, species r % 4): start, and the flat offsets
  int n = 0;
  if (tid < NR) {
    const int s = tid % kMaxTiledSpecies;
    const BrickCell c = brick_cell<TX, TY, TZ>(g, x0, y0, z0, tid / kMaxTiledSpecies);
    int b0 = 0;
    if (c.valid && s < args.ns) {
      const int32_t* cs = args.s[s].cell_start;
      b0 = cs[c.cell];
      n = cs[c.cell + 1] - b0;
    }
    rbeg[tid] = b0;
    rleft[tid] = 0;
  }
  int incl = n;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  if constexpr (MOVE) {
    for (int i = tid; i < 6 * HN; i += NT) {
      const int f = i / HN, nl = i % HN;
      const int gx = ((x0 - 1 + nl % HX) % g.nx + g.nx) % g.nx;
      const int gy = ((y0 - 1 + (nl / HX) % HY) % g.ny + g.ny) % g.ny;
      const int gz = ((z0 - 1 + nl / (HX * HY)) % g.nz + g.nz) % g.nz;
      const int64_t gn = (f % 3) * g.nn + gx + (int64_t)g.nx * (gy + (int64_t)g.ny * gz);
      fld[i] = f < 3 ? args.Emove[gn] : args.Bmove[gn];
    }
  }
  __syncthreads();
  {
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    if (tid < NR) roff[tid] = before + incl - n;
    if (tid == NR - 1) roff[NR] = before + incl;
  }
  __syncthreads();
  const int total = roff[NR];
  const bool mapped = total <= kMapCap;   // workgroup-uniform
  if (mapped && tid < NR) {
    const int a = roff[tid];
    for (int i = 0; i < n; ++i) rmap[a + i] = (uint8_t)tid;
  }
  __syncthreads();
  double kel = 0.0;
  WaveStrays<T> ws;
  WaveBuf<T>& wbuf = slist[wave];

  // flat index i -> (range, particle): from the map, else the last range with
  // roff <= i (the non-empty one holding i) by binary search
  auto locate = [&](int i, int& r) -> PData<T> {
    // Branch-free: a position past the list reads the last particle (never
    // stored back: ok is false), so every lane issues the same loads into
    // the same registers. Needs total > 0.
    PData<T> d;
    d.ok = i < total;
    const int ic = d.ok ? i : total - 1;
    int lo = 0;
    if (mapped) {   // workgroup-uniform
      lo = rmap[ic];
    } else {
      int hi = NR - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (roff[mid] <= ic) lo = mid;
        else hi = mid - 1;
      }
    }
    r = lo;
    const int s = lo % kMaxTiledSpecies;
    const int p = rbeg[lo] + (ic - roff[lo]);
    const TSpecies<T>& sp = lsp[s];
    d.s = s;
    d.p = p;
    d.x0 = gld(sp.pos[0] + p);
    d.x1 = gld(sp.pos[1] + p);
    d.x2 = gld(sp.pos[2] + p);
    d.v0 = gld(sp.vel[0] + p);
    d.v1 = gld(sp.vel[1] + p);
    d.v2 = gld(sp.vel[2] + p);
    // raw charge (0 for a constant-charge species, whose charge is added at
    // use): a select into the loaded register would make the compiler wait
    d.q = gld((sp.q ? sp.q : (const T*)args.zero) + (sp.q ? p : 0));
    if constexpr (sizeof(T) == 4) d.c = gld(sp.cell + p);
    else d.c = 0;
    return d;
  };

  // one particle per lane: move / check it and list it if it strays (reached
  // by the whole wavefront: the stray slots use ballots)
  auto process = [&](const PData<T>& pd, int r_cur) {
    // Branch-free: every lane runs the arithmetic and issues the same
    // stores (a lane without a particle writes into the sink block),
    // so the loop issues a fixed number of memory operations per iteration
    // and the next block's loads need not be waited for early.
    const TSpecies<T>& sp = lsp[pd.s];
    const T q = pd.q + (sp.q ? T(0) : sp.q_const);
    const BrickCell gc = brick_cell<TX, TY, TZ>(g, x0, y0, z0, r_cur / kMaxTiledSpecies);
    Stencil<T> ps = particle_stencil<T>(g, pd.x0, pd.x1, pd.x2, pd.c);
    const int pcell0 = ps.i[0] + g.nx * (ps.i[1] + g.ny * ps.i[2]);
    int item = (pd.s << kItemShift) | pd.p;
    // the listed state: the particle as it is now (moved, when moved here)
    SRec<T> rec{pd.x0, pd.x1, pd.x2, pd.v0, pd.v1, pd.v2, q, pd.c};
    bool stray;
    int lcell;
    if constexpr (MOVE) {
      // local cell in the halo'd box (periodic)
      const int dx = wrap_once(ps.i[0] - x0 + 1, g.nx);
      const int dy = wrap_once(ps.i[1] - y0 + 1, g.ny);
      const int dz = wrap_once(ps.i[2] - z0 + 1, g.nz);
      const bool inbox = pd.ok && dx <= TX + 1 && dy <= TY + 1 && dz <= TZ + 1;
      const int lx = inbox ? dx : 0, ly = inbox ? dy : 0, lz = inbox ? dz : 0;
      Vec3<T> Ep{T(0), T(0), T(0)}, Bp{T(0), T(0), T(0)};
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const T w = corner_weight(ps, a);
        const int nl = (lx + (a & 1)) + HX * ((ly + ((a >> 1) & 1)) + HY * (lz + ((a >> 2) & 1)));
        Ep.x = fma(w, fld[nl], Ep.x);
        Ep.y = fma(w, fld[HN + nl], Ep.y);
        Ep.z = fma(w, fld[2 * HN + nl], Ep.z);
        Bp.x = fma(w, fld[3 * HN + nl], Bp.x);
        Bp.y = fma(w, fld[4 * HN + nl], Bp.y);
        Bp.z = fma(w, fld[5 * HN + nl], Bp.z);
      }
      const Vec3<T> v = advance_velocity(Bp, sp.beta, Vec3<T>{pd.v0, pd.v1, pd.v2}, Ep);
      note_nonfinite(g, inbox && !(finite(v.x) && finite(v.y) && finite(v.z)));
      T n0, n1, n2;
      int pcell;
      if constexpr (sizeof(T) == 4) {
        int ix = ps.i[0], iy = ps.i[1], iz = ps.i[2];
        n0 = push_offset(ps.w1[0], v.x, args.dth[0], ix, g.nx);
        n1 = push_offset(ps.w1[1], v.y, args.dth[1], iy, g.ny);
        n2 = push_offset(ps.w1[2], v.z, args.dth[2], iz, g.nz);
        pcell = ix + g.nx * (iy + g.ny * iz);
      } else {
        n0 = push_abs(pd.x0, g.pdt[0], v.x, g.nx * g.hx);
        n1 = push_abs(pd.x1, g.pdt[1], v.y, g.ny * g.hy);
        n2 = push_abs(pd.x2, g.pdt[2], v.z, g.nz * g.hz);
        const Stencil<double> nps = stencil_abs(g, n0, n1, n2);
        pcell = nps.i[0] + g.nx * (nps.i[1] + g.ny * nps.i[2]);
      }
      // moved state in the box; unchanged beyond it (the stray mover moves it)
      if (inbox) {
        rec.x0 = n0;
        rec.x1 = n1;
        rec.x2 = n2;
        rec.v0 = v.x;
        rec.v1 = v.y;
        rec.v2 = v.z;
        rec.c = pcell;
      }
      const int wi = pd.ok ? pd.p : 0;
      T* const z = (T*)lsink;
      gst((pd.ok ? sp.pos[0] : z) + wi, rec.x0);
      gst((pd.ok ? sp.pos[1] : z) + wi, rec.x1);
      gst((pd.ok ? sp.pos[2] : z) + wi, rec.x2);
      gst((pd.ok ? sp.vel[0] : z) + wi, rec.v0);
      gst((pd.ok ? sp.vel[1] : z) + wi, rec.v1);
      gst((pd.ok ? sp.vel[2] : z) + wi, rec.v2);
      if constexpr (sizeof(T) == 4) gst((pd.ok ? sp.cell : (int32_t*)lsink) + wi, rec.c);
      if (args.ke) {
        const double vx = v.x, vy = v.y, vz = v.z;
        kel += inbox ? 0.5 * ((double)q * sp.inv_qom) * ((vx * vx + vy * vy) + vz * vz) : 0.0;
      }
      // listed: moved out of the range's cell, or beyond the box (unmoved)
      stray = pd.ok && (inbox ? pcell != gc.cell : true);
      if (pd.ok && !inbox) item |= kUnmoved;
      lcell = inbox ? pcell : gc.cell;
      if (args.stay && stray) atomicAdd(&rleft[r_cur], 1);
    } else {
      stray = pd.ok && pcell0 != gc.cell;
      lcell = pcell0;
    }
    ws.put(args, wbuf, lane, stray, item, lcell, rec);
  };

  if (total == 0) {
    // no particles in the brick: nothing to move or list
  } else if constexpr (sizeof(T) == 4) {
    // two blocks of 64 per wavefront and iteration, the next two blocks'
    // loads in flight while these are processed
    int ra, rb;
    PData<T> pa = locate(wave * 128 + lane, ra);
    PData<T> pb = locate(wave * 128 + 64 + lane, rb);
    // the first blocks are waited for here, so that at the loop head no
    // load from before the loop is pending (else the compiler waits for all
    // loads, the next blocks' included, at the first use)
    __builtin_amdgcn_s_waitcnt(0);
    // unrolled once more, so that the two register sets swap roles instead
    // of being copied (a copy of a loaded register waits for its load)
    int rna, rnb;
    PData<T> na, nb;
    for (int base = wave * 128; base < total;) {
      na = locate(base + 2 * NT + lane, rna);
      nb = locate(base + 2 * NT + 64 + lane, rnb);
      process(pa, ra);
      process(pb, rb);
      base += 2 * NT;
      if (base >= total) break;   // workgroup-uniform
      pa = locate(base + 2 * NT + lane, ra);
      pb = locate(base + 2 * NT + 64 + lane, rb);
      process(na, rna);
      process(nb, rnb);
      base += 2 * NT;
    }
  } else {
    // FP64: one block per iteration (its registers allow no second)
    int ra, rna;
    PData<T> pa = locate(wave * 64 + lane, ra), na;
    for (int base = wave * 64; base < total;) {
      na = locate(base + NT + lane, rna);
      process(pa, ra);
      base += NT;
      if (base >= total) break;
      pa = locate(base + NT + lane, ra);
      process(na, rna);
      base += NT;
    }
  }
  if constexpr (MOVE) {
    if (args.ke) {
      for (int off = 32; off > 0; off >>= 1) kel += __shfl_down(kel, off);
      if (lane == 0) red[wave] = kel;
    }
  }
  // the strays still held take one reservation of the workgroup in the list
  if (lane == 0) wst[wave] = ws.fill;
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
    for (int w = 0; w < NW; ++w) tot += wst[w];
    int b = tot ? atomicAdd(args.stray_count, tot) : 0;
    for (int w = 0; w < NW; ++w) {
      const int c = wst[w];
      wst[w] = b;
      b += c;
    }
    if constexpr (MOVE) {
      if (args.ke) {
        double s = 0.0;
        for (int w = 0; w < NW; ++w) s += red[w];
        if (s != 0.0) unsafeAtomicAdd(args.ke, s);
      }
    }
  }
  __syncthreads();
  if (MOVE && args.stay && tid < NR) {
    const int s = tid % kMaxTiledSpecies;
    const BrickCell c = brick_cell<TX, TY, TZ>(g, x0, y0, z0, tid / kMaxTiledSpecies);
    if (c.valid && s < args.ns) args.stay[(int64_t)s * g.nn + c.cell] = roff[tid + 1] - roff[tid] - rleft[tid];
  }
  ws.copy_out(args, wbuf, lane, wst[wave]);
}
// ---------------------------------------------------------------------------
// grouped mover
// ---------------------------------------------------------------------------
// A workgroup owns a brick of TX x TY x TZ cells. It stages the mover fields
// E^{n+theta}, B^n on the brick's nodes plus a one-cell halo in LDS, one
// record of (E, B) per node so that a corner is two 16-byte reads, then its
// wavefronts run through the brick's particles species by species: the
// species' cell ranges of the brick, taken as one list padded to whole blocks
// of 64, so that every block belongs to one species and reads and writes its
// arrays through buffer resources in scalar registers with one 32-bit offset
// per lane (a lane past the list has an offset beyond the buffer: its loads
// read zero, its stores are dropped). The next block's loads are in flight
// while a block is moved. A particle whose cell lies in the halo'd box is
// moved with the staged fields (the same gathers, rotation and push as every
// other mover) and written back, and listed if it is now outside its range's
// cell; a particle beyond the box is listed unmoved (with its range's cell)
// for the stray mover.
template <typename T>
struct MoverRsrc {
  __amdgpu_buffer_rsrc_t pos[3], vel[3], q, cell;
};

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* p, int64_t bytes) {
  // raw buffer: stride 0, range checked against the byte count
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0,
                                           (int)(bytes < 0x7fffffff ? bytes : 0x7fffffff), 0x00020000);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
}
template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, T v) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
  }
}

// one particle's inputs of the grouped mover, loaded ahead of use
template <typename T>
struct MData {
  T x0, x1, x2, v0, v1, v2, q;
  int c;      // stored cell (FP32 form)
  int lc;     // local cell of its range
  int p;      // index in the species arrays
  bool ok;
};

template <typename T, int TX, int TY, int TZ, int NW>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
k_mover(Grid g, TArgs<T> args, int ntx, int nty, int ntz) {
  constexpr int NCELL = TX * TY * TZ;
  constexpr int HX = TX + 3, HY = TY + 3, HZ = TZ + 3, HN = HX * HY * HZ;   // halo'd node box
  constexpr int NT = NW * 64;
  constexpr int NS = kMaxTiledSpecies;
  static_assert(NS * NCELL <= NT, "one range per thread");
  // per node: Ex Ey Ez Bx By Bz and two pad values (16-byte aligned halves)
  __shared__ __attribute__((aligned(16))) T fld[HN * 8];
  __shared__ int rbeg[NS * NCELL];        // range (species s, cell lc) at s * NCELL + lc
  __shared__ int roff[NS * (NCELL + 1)];  // species s: list offsets of its cells, [s][lc]
  __shared__ int rleft[NS * NCELL];       // regrouping: particles of each range listed as strays
  __shared__ int sblk[NS + 1];            // first block of each species in the workgroup's block order
  __shared__ double red[NW];
  __shared__ int wst[NW];
  __shared__ WaveBuf<T> slist[NW];
  __shared__ uint8_t rmap[kMapCap];       // list position -> local cell, per species (when it fits)
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int x0, y0, z0;
  brick_origin<TX, TY, TZ>(ntx, nty, ntz, x0, y0, z0);
  const int ns = args.ns;

  // ranges: thread t = s * NCELL + lc
  int n = 0;
  if (tid < NS * NCELL) {
    const int s = tid / NCELL, lc = tid % NCELL;
    const BrickCell c = brick_cell<TX, TY, TZ>(g, x0, y0, z0, lc);
    int b0 = 0;
    if (c.valid && s < ns) {
      const int32_t* cs = args.s[s].cell_start;
      b0 = cs[c.cell];
      n = cs[c.cell + 1] - b0;
    }
    rbeg[tid] = b0;
    rleft[tid] = 0;
  }
  // per-species exclusive scan over the NCELL cells (NCELL = 32: within half
  // a wavefront)
  static_assert(NCELL <= 64 && 64 % NCELL == 0, "a species' cells within one wavefront");
  int incl = n;
#pragma unroll
  for (int o = 1; o < NCELL; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if ((lane % NCELL) >= o) incl += y;
  }
  if (tid < NS * NCELL) {
    const int s = tid / NCELL, lc = tid % NCELL;
    roff[s * (NCELL + 1) + lc] = incl - n;
    if (lc == NCELL - 1) roff[s * (NCELL + 1) + NCELL] = incl;
  }
  for (int nl = tid; nl < HN; nl += NT) {
    // any number of periods: a dimension may hold fewer cells than the box
    const int gx = ((x0 - 1 + nl % HX) % g.nx + g.nx) % g.nx;
    const int gy = ((y0 - 1 + (nl / HX) % HY) % g.ny + g.ny) % g.ny;
    const int gz = ((z0 - 1 + nl / (HX * HY)) % g.nz + g.nz) % g.nz;
    const int64_t gn = gx + (int64_t)g.nx * (gy + (int64_t)g.ny * gz);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      fld[8 * nl + f] = args.Emove[f * g.nn + gn];
      fld[8 * nl + 3 + f] = args.Bmove[f * g.nn + gn];
    }
    fld[8 * nl + 6] = T(0);
    fld[8 * nl + 7] = T(0);
  }
  __syncthreads();
  if (tid == 0) {
    int b = 0;
    for (int s = 0; s < NS; ++s) {
      sblk[s] = b;
      b += (roff[s * (NCELL + 1) + NCELL] + 63) >> 6;
    }
    sblk[NS] = b;
  }
  // the list position -> cell map of each species, if every species' list fits
  int tmax = 0;
  for (int s = 0; s < NS; ++s) {
    const int t = roff[s * (NCELL + 1) + NCELL];
    tmax = t > tmax ? t : tmax;
  }
  const bool mapped = tmax * ns <= kMapCap;   // workgroup-uniform (the species in use)
  const int mstride = mapped ? tmax : 0;
  if (mapped && tid < NS * NCELL) {
    const int s = tid / NCELL, lc = tid % NCELL;
    const int a = roff[s * (NCELL + 1) + lc];
    for (int i = 0; i < n; ++i) rmap[s * mstride + a + i] = (uint8_t)lc;
  }
  __syncthreads();
  const int nblk = sblk[NS];

  // the species' arrays as buffers (scalar registers)
  auto rsrc_of = [&](int s) {
    MoverRsrc<T> R;
    const TSpecies<T>& sp = args.s[s];
    const int64_t np = sp.np;
    for (int d = 0; d < 3; ++d) {
      R.pos[d] = buffer_of<T>(sp.pos[d], np * (int64_t)sizeof(T));
      R.vel[d] = buffer_of<T>(sp.vel[d], np * (int64_t)sizeof(T));
    }
    R.q = buffer_of<T>(sp.q ? (const void*)sp.q : args.zero, sp.q ? np * (int64_t)sizeof(T) : 0);
    R.cell = buffer_of<T>(sp.cell ? (const void*)sp.cell : args.zero, sp.cell ? np * 4 : 0);
    return R;
  };

  // block b of the workgroup's order: species s, lane position i in its list
  auto load = [&](int b, int& s_out) -> MData<T> {
    int s = 0;
#pragma unroll
    for (int k = 1; k < NS; ++k) s += b >= sblk[k] ? 1 : 0;
    s = __builtin_amdgcn_readfirstlane(s);
    s_out = s;
    const int i = (b - sblk[s]) * 64 + lane;
    const int* ro = roff + s * (NCELL + 1);
    const int tot = ro[NCELL];
    MData<T> d;
    d.ok = i < tot;
    const int ic = d.ok ? i : tot - 1;
    int lc;
    if (mapped) {   // workgroup-uniform
      lc = rmap[s * mstride + ic];
    } else {
      lc = 0;
#pragma unroll
      for (int step = NCELL / 2; step > 0; step >>= 1) lc += ro[lc + step] <= ic ? step : 0;
    }
    d.lc = lc;
    d.p = rbeg[s * NCELL + lc] + (ic - ro[lc]);
    const uint32_t off = d.ok ? (uint32_t)d.p * (uint32_t)sizeof(T) : 0xffffffffu;
    const MoverRsrc<T> R = rsrc_of(s);
    d.x0 = bload<T>(R.pos[0], off);
    d.x1 = bload<T>(R.pos[1], off);
    d.x2 = bload<T>(R.pos[2], off);
    d.v0 = bload<T>(R.vel[0], off);
    d.v1 = bload<T>(R.vel[1], off);
    d.v2 = bload<T>(R.vel[2], off);
    d.q = bload<T>(R.q, off);   // 0 for a constant-charge species (empty buffer)
    d.c = sizeof(T) == 4 ? (int)__builtin_amdgcn_raw_buffer_load_b32(R.cell, d.ok ? (uint32_t)d.p * 4u : 0xffffffffu, 0, 0) : 0;
    return d;
  };

  double kel = 0.0;
  WaveStrays<T> ws;
  WaveBuf<T>& wbuf = slist[wave];

  auto process = [&](const MData<T>& pd, int s) {
    const TSpecies<T>& sp = args.s[s];
    const T q = pd.q + (sp.q ? T(0) : sp.q_const);
    const BrickCell gc = brick_cell<TX, TY, TZ>(g, x0, y0, z0, pd.lc);
    const Stencil<T> ps = particle_stencil<T>(g, pd.x0, pd.x1, pd.x2, pd.c);
    int item = (s << kItemShift) | pd.p;
    SRec<T> rec{pd.x0, pd.x1, pd.x2, pd.v0, pd.v1, pd.v2, q, pd.c};
    // local cell in the halo'd box (periodic)
    const int dx = wrap_once(ps.i[0] - x0 + 1, g.nx);
    const int dy = wrap_once(ps.i[1] - y0 + 1, g.ny);
    const int dz = wrap_once(ps.i[2] - z0 + 1, g.nz);
    const bool inbox = pd.ok && dx <= TX + 1 && dy <= TY + 1 && dz <= TZ + 1;
    const int lx = inbox ? dx : 0, ly = inbox ? dy : 0, lz = inbox ? dz : 0;
    const T* const fb = fld + 8 * (lx + HX * (ly + HY * lz));
    Vec3<T> Ep{T(0), T(0), T(0)}, Bp{T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const T w = corner_weight(ps, a);
      const T* const f = fb + 8 * ((a & 1) + HX * (((a >> 1) & 1) + HY * ((a >> 2) & 1)));
      Ep.x = fma(w, f[0], Ep.x);
      Ep.y = fma(w, f[1], Ep.y);
      Ep.z = fma(w, f[2], Ep.z);
      Bp.x = fma(w, f[3], Bp.x);
      Bp.y = fma(w, f[4], Bp.y);
      Bp.z = fma(w, f[5], Bp.z);
    }
    const Vec3<T> v = advance_velocity(Bp, sp.beta, Vec3<T>{pd.v0, pd.v1, pd.v2}, Ep);
    note_nonfinite(g, inbox && !(finite(v.x) && finite(v.y) && finite(v.z)));
    T n0, n1, n2;
    int pcell;
    if constexpr (sizeof(T) == 4) {
      int ix = ps.i[0], iy = ps.i[1], iz = ps.i[2];
      n0 = push_offset(ps.w1[0], v.x, args.dth[0], ix, g.nx);
      n1 = push_offset(ps.w1[1], v.y, args.dth[1], iy, g.ny);
      n2 = push_offset(ps.w1[2], v.z, args.dth[2], iz, g.nz);
      pcell = ix + g.nx * (iy + g.ny * iz);
    } else {
      n0 = push_abs(pd.x0, g.pdt[0], v.x, g.nx * g.hx);
      n1 = push_abs(pd.x1, g.pdt[1], v.y, g.ny * g.hy);
      n2 = push_abs(pd.x2, g.pdt[2], v.z, g.nz * g.hz);
      const Stencil<double> nps = stencil_abs(g, n0, n1, n2);
      pcell = nps.i[0] + g.nx * (nps.i[1] + g.ny * nps.i[2]);
    }
    // moved state in the box; unchanged beyond it (the stray mover moves it)
    if (inbox) {
      rec.x0 = n0;
      rec.x1 = n1;
      rec.x2 = n2;
      rec.v0 = v.x;
      rec.v1 = v.y;
      rec.v2 = v.z;
      rec.c = pcell;
    }
    // write back: lanes without a particle have an offset past the buffer
    const uint32_t off = pd.ok ? (uint32_t)pd.p * (uint32_t)sizeof(T) : 0xffffffffu;
    const MoverRsrc<T> R = rsrc_of(s);
    bstore<T>(R.pos[0], off, rec.x0);
    bstore<T>(R.pos[1], off, rec.x1);
    bstore<T>(R.pos[2], off, rec.x2);
    bstore<T>(R.vel[0], off, rec.v0);
    bstore<T>(R.vel[1], off, rec.v1);
    bstore<T>(R.vel[2], off, rec.v2);
    if constexpr (sizeof(T) == 4)
      __builtin_amdgcn_raw_buffer_store_b32((uint32_t)rec.c, R.cell, pd.ok ? (uint32_t)pd.p * 4u : 0xffffffffu, 0, 0);
    if (args.ke) {
      const double vx = v.x, vy = v.y, vz = v.z;
      kel += inbox ? 0.5 * ((double)q * sp.inv_qom) * ((vx * vx + vy * vy) + vz * vz) : 0.0;
    }
    // listed: moved out of the range's cell, or beyond the box (unmoved)
    const bool stray = pd.ok && (inbox ? pcell != gc.cell : true);
    if (pd.ok && !inbox) item |= kUnmoved;
    const int lcell = inbox ? pcell : gc.cell;
    if (args.stay && stray) atomicAdd(&rleft[s * NCELL + pd.lc], 1);
    ws.put(args, wbuf, lane, stray, item, lcell, rec);
  };

  // blocks wave, wave + NW, ...: the next block's loads in flight while one
  // is moved; unrolled once so that the two register sets swap roles (a copy
  // of a loaded register would wait for its load)
  if (wave < nblk) {
    int sa, sb;
    MData<T> pa = load(wave, sa), pb;
    for (int b = wave; b < nblk;) {
      const bool nb1 = b + NW < nblk;
      if (nb1) pb = load(b + NW, sb);
      process(pa, sa);
      b += NW;
      if (!nb1) break;
      const bool nb2 = b + NW < nblk;
      if (nb2) pa = load(b + NW, sa);
      process(pb, sb);
      b += NW;
      if (!nb2) break;
    }
  }
  if (args.ke) {
    for (int off = 32; off > 0; off >>= 1) kel += __shfl_down(kel, off);
    if (lane == 0) red[wave] = kel;
  }
  // the strays still held take one reservation of the workgroup in the list
  if (lane == 0) wst[wave] = ws.fill;
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
    for (int w = 0; w < NW; ++w) tot += wst[w];
    int b = tot ? atomicAdd(args.stray_count, tot) : 0;
    for (int w = 0; w < NW; ++w) {
      const int c = wst[w];
      wst[w] = b;
      b += c;
    }
    if (args.ke) {
      double sum = 0.0;
      for (int w = 0; w < NW; ++w) sum += red[w];
      if (sum != 0.0) unsafeAtomicAdd(args.ke, sum);
    }
  }
  __syncthreads();
  if (args.stay && tid < NS * NCELL) {
    const int s = tid / NCELL, lc = tid % NCELL;
    const BrickCell c = brick_cell<TX, TY, TZ>(g, x0, y0, z0, lc);
    if (c.valid && s < ns)
      args.stay[(int64_t)s * g.nn + c.cell] =
          roff[s * (NCELL + 1) + lc + 1] - roff[s * (NCELL + 1) + lc] - rleft[tid];
  }
  ws.copy_out(args, wbuf, lane, wst[wave]);
}

// ---------------------------------------------------------------------------
// tiled deposit
// ---------------------------------------------------------------------------
// A workgroup owns a brick of cells and stages B at the brick's nodes in
// LDS; each wavefront takes the brick's cells one at a time. Per cell the
// wavefront-uniform quantities (the cell's particle ranges, the regrouping
// starts) are loaded one cell ahead, one value per lane, and moved to scalar
// registers; each block of 64 list positions is one particle per lane:
//   1. the lane's record (12 values, 27 class weights) goes to LDS;
//   2. the next block's loads are issued (this cell's, else the next cell's);
//   3. 16 matrix-core steps of K = 4 particles reduce the block, from zero,
//      and the block sum is added to the cell's running sums (FP32: Kahan).
// At the end of a cell its class sums and corner currents are written to the
// per-cell sums in global memory; the node flush then forms J and M.
// With REGROUP the deposit also writes every particle it takes (the cell's own
// range particles still in the cell, then its strays) to the targets, species
// by species in cell order: the next pass's grouping, without a separate sort.
// FP32: 5 waves per SIMD (96 VGPRs, a few spilled: 709 -> 676 us at 64^3),
// 4 for the regrouping form, which spills more at 5 (900 -> 930 us)
template <typename T, int TX, int TY, int TZ, int NW, bool REGROUP>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (REGROUP ? 4 : 5) : 1)))
k_deposit(Grid g, TArgs<T> args, int ntx, int nty, int ntz) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc;
  constexpr int NCELL = TX * TY * TZ;
  constexpr int WREC = kRows * kSlots;
  constexpr int NX = TX + 1, NY = TY + 1, NZ = TZ + 1, NBN = NX * NY * NZ;   // brick nodes
  // the wavefront records, and two rows more: the matrix-core operand reads
  // of the unused classes 27-31 reach two rows past a wavefront's records
  __shared__ __attribute__((aligned(16))) T smem[NW * WREC + 2 * kSlots];
  __shared__ __attribute__((aligned(16))) T bst[NBN * 4];   // B at the brick's nodes: x, y, z, pad
  __shared__ TSpecies<T> lsp[kMaxTiledSpecies];
  __shared__ PtrSet<T> lptr_tab[kZeroSlot + 1];
  // regrouping targets, read from LDS where used (kept in scalar registers
  // they would crowd out the cell's uniform values)
  __shared__ RegroupDst<T> ldst[REGROUP ? kMaxTiledSpecies : 1];
  LdsPtrSet<T>* const lptr = (LdsPtrSet<T>*)lptr_tab;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = lane & 15;   // MFMA column (class) of this lane
  const int grp = lane >> 4;   // MFMA k-group of this lane
  int x0, y0, z0;
  brick_origin<TX, TY, TZ>(ntx, nty, ntz, x0, y0, z0);

  for (int i = tid; i < NW * WREC + 2 * kSlots; i += NW * 64) smem[i] = T(0);
  fill_tables(args, lsp, lptr_tab, tid);
  for (int nl = tid; nl < NBN; nl += NW * 64) {
    const int gx = (x0 + nl % NX) % g.nx, gy = (y0 + (nl / NX) % NY) % g.ny, gz = (z0 + nl / (NX * NY)) % g.nz;
    const int64_t gn = gx + (int64_t)g.nx * (gy + (int64_t)g.ny * gz);
#pragma unroll
    for (int c = 0; c < 3; ++c) bst[4 * nl + c] = args.Bdep[c * g.nn + gn];
    bst[4 * nl + 3] = T(0);
  }
  if constexpr (REGROUP) {
#pragma unroll
    for (int k = 0; k < kMaxTiledSpecies; ++k)
      if (tid == 8 + k) ldst[k] = args.dst[k < args.ns ? k : 0];
  }
  __syncthreads();

  T* const wrec = smem + wave * WREC;
  const T* const opnd = wrec + col * kSlots + grp;   // row col, slot grp
  // this lane's classes: col in tile 0, 15 + col in tile 1 (classes 15-30:
  // the same x factor, the y-z product 5 rows on; class 15 is taken from
  // tile 0 and 27-30 are not used)
  const T* const fx0 = wrec + (12 + col % 3) * kSlots + grp;
  const T* const fq0 = wrec + (15 + col / 3) * kSlots + grp;
  T* const tcur = wrec + kTcur;                       // current class sums [27][3]

  // One-cell-ahead loads, one value per lane: lanes 0..9 the cell's range
  // bounds (lo, hi of slot l / 2), lanes 0..3 the regrouping starts.
  auto load_cell = [&](const BrickCell& c, int& rv, int& dv) {
    rv = 0;
    dv = 0;
    const int cl = c.valid ? c.cell : 0;
    if (lane < 2 * kSlots5) {
      const int s = lane >> 1;
      const int32_t* cs = s == kStraySlot ? args.ind_start : lsp[s < kMaxTiledSpecies ? s : 0].cell_start;
      rv = gld(cs + cl + (lane & 1));
    }
    if constexpr (REGROUP) {
      if (lane < kMaxTiledSpecies) dv = gld(ldst[lane].start + cl);
    }
  };
  // the cell's ranges from the loaded bounds (wavefront-uniform)
  auto cell_ranges = [&](const BrickCell& c, int rv) -> Ranges {
    RangeLd r;
#pragma unroll
    for (int s = 0; s < kSlots5; ++s) {
      r.lo[s] = __builtin_amdgcn_readlane(rv, 2 * s);
      r.hi[s] = __builtin_amdgcn_readlane(rv, 2 * s + 1);
    }
    return make_ranges<T, kSlots5>(args, r, c);
  };

  BrickCell cc = brick_cell<TX, TY, TZ>(g, x0, y0, z0, wave);
  int rv, dv;
  load_cell(cc, rv, dv);
  Ranges cr = cell_ranges(cc, rv);
  PData<T> pd = load_dep<T>(lptr, cr, lane);

  for (int lc = wave; lc < NCELL; lc += NW) {
    const bool has_next = lc + NW < NCELL;   // wave-uniform
    const BrickCell nc = brick_cell<TX, TY, TZ>(g, x0, y0, z0, has_next ? lc + NW : lc);
    // this cell's regrouping starts, in scalar registers, and its corners'
    // B in LDS
    int dst0[kMaxTiledSpecies];
#pragma unroll
    for (int s = 0; s < kMaxTiledSpecies; ++s) dst0[s] = REGROUP ? __builtin_amdgcn_readlane(dv, s) : 0;
    const T* const nb = bst + 4 * ((lc % TX) + NX * ((lc / TX) % TY + NY * (lc / (TX * TY))));
    // the next cell's, in flight while this cell is processed
    int nrv = 0, ndv = 0;
    if (has_next) load_cell(nc, nrv, ndv);

    const int cell = cc.cell;   // -1: not a cell of the grid (a clipped brick)
    const int cnt = cr.total;   // wave-uniform
    if (cnt == 0) {
      if (cell >= 0)
        for (int i = lane; i < SCS; i += 64) gst(args.csum + (int64_t)cell * SCS + i, T(0));
      if (has_next) {
        cr = cell_ranges(nc, nrv);
        pd = load_dep<T>(lptr, cr, lane);
      }
      cc = nc;
      rv = nrv;
      dv = ndv;
      continue;
    }
    int run[kMaxTiledSpecies] = {0, 0, 0, 0};   // regrouping: particles written per species
    T S[2][4], C[2][4];                         // running sums [tile][reg]
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) { S[t][r] = T(0); C[t][r] = T(0); }

    for (int cb = 0; cb < cnt; cb += 64) {
      // ---- 1. this lane's record; lanes without a particle of the cell
      // (past the count, or no longer in the cell) carry zero charge ----
      bool keep;
      {
        const TSpecies<T>& sp = lsp[dep_species(pd)];
        const Stencil<T> ps = particle_stencil<T>(g, pd.x0, pd.x1, pd.x2, pd.c);
        if constexpr (sizeof(T) == 4) keep = pd.ok && pd.c == cell;
        else keep = pd.ok && ps.i[0] + g.nx * (ps.i[1] + g.ny * ps.i[2]) == cell;
        T W[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) W[a] = corner_weight(ps, a);
        // B at the position from the cell's corners (the mover's order of
        // accumulation, so the two agree bit for bit in FP64)
        Vec3<T> B1{T(0), T(0), T(0)};
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const T* const f = nb + 4 * ((a & 1) + NX * (((a >> 1) & 1) + NY * ((a >> 2) & 1)));
          B1.x = fma(W[a], f[0], B1.x);
          B1.y = fma(W[a], f[1], B1.y);
          B1.z = fma(W[a], f[2], B1.z);
        }
        T r[kRec];
        particle_record(ps, B1, Vec3<T>{pd.v0, pd.v1, pd.v2}, keep ? dep_charge(pd, lptr) : T(0), sp, r);
#pragma unroll
        for (int i = 0; i < kRec; ++i) wrec[i * kSlots + lane] = r[i];
      }
      if constexpr (REGROUP) {
        // species by species (a block mostly holds one): the target index is
        // the cell's start for the species, the particles of the species
        // written so far in this cell, and the lanes before this one taking
        // the same species
        const int sl = dep_species(pd);
        const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
        for (int s = 0; s < kMaxTiledSpecies; ++s) {
          if (s < args.ns) {   // wave-uniform
            const bool mine = keep && sl == s;
            const uint64_t m = __ballot(mine);
            const int my = dst0[s] + run[s] + __popcll(m & below);
            run[s] += __popcll(m);
            if (m) {   // wave-uniform
              const RegroupDst<T>& D = ldst[s];
              if (mine && my >= 0 && my < D.np) {
                gst(D.pos[0] + my, pd.x0);
                gst(D.pos[1] + my, pd.x1);
                gst(D.pos[2] + my, pd.x2);
                gst(D.vel[0] + my, pd.v0);
                gst(D.vel[1] + my, pd.v1);
                gst(D.vel[2] + my, pd.v2);
                if (D.q) gst(D.q + my, pd.q);   // a per-particle charge: its raw load is the charge
                if constexpr (sizeof(T) == 4) gst(D.cell + my, pd.c);
              }
            }
          }
        }
      }
      wave_sync();
      // ---- 2. the next block's loads (this cell's, else the next cell's
      // first), in flight while this block is reduced ----
      const bool same = cb + 64 < cnt;   // wave-uniform
      if (!same && has_next) cr = cell_ranges(nc, nrv);
      pd = load_dep<T>(lptr, cr, same ? cb + 64 + lane : lane);
      // ---- 3. matrix cores: block sums [value][class] from zero; the steps
      // past the cell's count are skipped (their records are zero) ----
      const int nk = cnt - cb;   // wave-uniform, >= 1
      acc_t d0 = {0, 0, 0, 0}, d1 = {0, 0, 0, 0};
#pragma unroll
      for (int k4 = 0; k4 < 64; k4 += 4) {
        if (k4 > 0 && k4 >= nk) break;
        const T a = opnd[k4];
        const T fx = fx0[k4];
        const T b0 = fx * fq0[k4];
        const T b1 = fx * fq0[5 * kSlots + k4];
        d0 = MF::run(a, b0, d0);
        d1 = MF::run(a, b1, d1);
      }
      if (cb == 0) {
        // the cell's first block: the compensated sum of one term is the term
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          S[0][q] = d0[q];
          S[1][q] = d1[q];
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if constexpr (sizeof(T) == 4) {
            kahan(S[0][q], C[0][q], d0[q]);
            kahan(S[1][q], C[1][q], d1[q]);
          } else {
            S[0][q] += d0[q];
            S[1][q] += d1[q];
          }
        }
      }
      wave_sync();
    }

    // ---- per-cell sums to global memory: the mass-matrix classes; the
    // current classes to LDS, from which the corner currents follow ----
    T* const sc = args.csum + (int64_t)(cell >= 0 ? cell : 0) * SCS;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int cls = t * 15 + col;
      if (cls >= 27 || (t == 1 && col == 0)) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = MF::row(lane, q);
        T v = S[t][q];
        if constexpr (sizeof(T) == 4) v -= C[t][q];
        if (row < 9) {
          if (cell >= 0) gst(sc + cls * 9 + row, v);
        } else if (row < 12) {
          tcur[cls * 3 + (row - 9)] = v;
        }
      }
    }
    wave_sync();
    // corner currents J_a = sum_b T_{a+b}: lanes 0..23
    if (lane < 24 && cell >= 0) {
      const int a = lane / 3, comp = lane % 3;
      const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      T s = T(0);
#pragma unroll
      for (int bb = 0; bb < 8; ++bb) {
        const int cls = (ax + (bb & 1)) + 3 * (ay + ((bb >> 1) & 1)) + 9 * (az + ((bb >> 2) & 1));
        s += tcur[cls * 3 + comp];
      }
      gst(sc + 243 + 3 * a + comp, s);
    }
    wave_sync();
    cc = nc;
    rv = nrv;
    dv = ndv;
  }
}

// ---------------------------------------------------------------------------
// node flush: every node's J and 14 mass-matrix blocks from the per-cell sums
// ---------------------------------------------------------------------------
// Node g is corner a of the 8 cells g - a. Block k of g holds every stored
// pair (a, a + o_k) of those cells, whose weight class 2a + o_k picks the
// cell's class sum; the current at g is the sum of the cells' corner-a
// currents. A workgroup owns a brick of FX x FY x FZ nodes: it stages the
// per-cell sums of the (FX+1)(FY+1)(FZ+1) cells around them in LDS (each
// cell's sums are contiguous, so the loads coalesce), then every (entry,
// node) adds its at most 8 terms in FP64 and stores the rounded result once
// (with accumulate: added to J and M). Every node has one owner: no atomics,
// and J and M need no clearing.
template <typename T, int FX, int FY, int FZ, int NT>
__global__ void __launch_bounds__(NT) k_flush_nodes(Grid g, const T* __restrict__ csum, T* __restrict__ J,
                                                     T* __restrict__ M, int accumulate, int nbx, int nby, int nbz) {
  constexpr int CX = FX + 1, CY = FY + 1, CZ = FZ + 1, NC = CX * CY * CZ;
  constexpr int NN = FX * FY * FZ;
  // staged cells SL apart: an odd stride puts the same entry of neighbouring
  // cells (the lanes' nodes) in distinct LDS banks
  constexpr int SL = SCS + 1;
  __shared__ T rec[NC * SL];
  __shared__ int64_t cbase[NC];
  int x0, y0, z0;
  brick_origin<FX, FY, FZ>(nbx, nby, nbz, x0, y0, z0);
  const int tid = threadIdx.x;
  // cell c = (x0 - 1 + cx, y0 - 1 + cy, z0 - 1 + cz), periodic (any number
  // of periods: a dimension may hold fewer cells than the brick)
  if (tid < NC) {
    const int cx = ((x0 - 1 + tid % CX) % g.nx + g.nx) % g.nx;
    const int cy = ((y0 - 1 + (tid / CX) % CY) % g.ny + g.ny) % g.ny;
    const int cz = ((z0 - 1 + tid / (CX * CY)) % g.nz + g.nz) % g.nz;
    cbase[tid] = (cx + (int64_t)g.nx * (cy + (int64_t)g.ny * cz)) * SCS;
  }
  __syncthreads();
  // staged 16 values per thread at a time, all loads in flight together
  constexpr int TOT = NC * SCS, CH = 16;
  for (int i0 = 0; i0 < TOT; i0 += NT * CH) {
    T v[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int i = i0 + j * NT + tid;
      const int ic = i < TOT ? i : TOT - 1;
      const int c = ic / SCS, e = ic - c * SCS;
      v[j] = csum[cbase[c] + e];
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int i = i0 + j * NT + tid;
      const int c = i / SCS;
      if (i < TOT) rec[i + c] = v[j];   // c * SL + (i - c * SCS)
    }
  }
  __syncthreads();
  bool bad = false;
  auto put = [&](T* o, double v) {
    const T out = accumulate ? (T)((double)*o + v) : (T)v;
    bad = bad || !finite(out);
    *o = out;
  };
  // items (group, node): groups 0..8 the mass-matrix entry ij of all 14
  // blocks, group 9 the three current components
  for (int it = tid; it < 10 * NN; it += NT) {
    const int grp = it / NN, ln = it - grp * NN;
    const int lx = ln % FX, ly = (ln / FX) % FY, lz = ln / (FX * FY);
    const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
    if (gx >= g.nx || gy >= g.ny || gz >= g.nz) continue;   // a clipped brick
    const int64_t gn = gx + (int64_t)g.nx * (gy + (int64_t)g.ny * gz);
    // the staged cell g - a is (lx + 1 - ax, ly + 1 - ay, lz + 1 - az)
    const T* const cb = rec + ((lx + 1) + CX * ((ly + 1) + CY * (lz + 1))) * SL;
    if (grp < 9) {
      const int ij = grp;
#pragma unroll
      for (int k = 0; k < 14; ++k) {
        double v = 0.0;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const int cls = pair_class(k, a);
          if (cls < 0) continue;
          const int off = (a & 1) + CX * (((a >> 1) & 1) + CY * ((a >> 2) & 1));
          v += (double)cb[-off * SL + cls * 9 + ij];
        }
        put(M + (int64_t)(k * 9 + ij) * g.nn + gn, v);
      }
    } else {
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        double v = 0.0;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const int off = (a & 1) + CX * (((a >> 1) & 1) + CY * ((a >> 2) & 1));
          v += (double)cb[-off * SL + 243 + 3 * a + comp];
        }
        put(J + (int64_t)comp * g.nn + gn, v);
      }
    }
  }
  note_nonfinite(g, bad);
}

// ---------------------------------------------------------------------------
// diagnostic moments over cell-grouped particles (Sec. III, diagnostics for
// I/O): per cell, the 10 particle values f = q (1, v, v_i v_j) against the 8
// corner weights are a (10 x K) by (K x 8) contraction over the cell's K
// particles, one 16 x 16 matrix-core tile per cell (rows past 10 and columns
// past 8 are not used); per-cell sums go to LDS and a node gather adds each
// brick node once to the global arrays. A particle not in its range's cell
// (stale grouping) is added with global atomics instead.
// ---------------------------------------------------------------------------
constexpr int kDVals = 10;                  // q, q v (3), q v_i v_j (xx xy xz yy yz zz)
constexpr int kDRows = kDVals + 16;         // values, then 8 weights (+8 rows read as unused columns)
constexpr int kDCell = kDVals * 8;          // per-cell sums: [value][corner]

template <typename T>
__device__ __forceinline__ void diag_values(T q, T vx, T vy, T vz, T f[kDVals]) {
  f[0] = q;
  f[1] = q * vx;
  f[2] = q * vy;
  f[3] = q * vz;
  f[4] = (q * vx) * vx;
  f[5] = (q * vx) * vy;
  f[6] = (q * vx) * vz;
  f[7] = (q * vy) * vy;
  f[8] = (q * vy) * vz;
  f[9] = (q * vz) * vz;
}

template <typename T>
__device__ __forceinline__ T* diag_target(T* rho, T* Jd, T* P, int64_t nn, int v, int64_t node) {
  return v == 0 ? rho + node : (v < 4 ? Jd + (v - 1) * nn + node : P + (v - 4) * nn + node);
}

template <typename T, int TX, int TY, int TZ, int NW>
__global__ void __launch_bounds__(NW * 64) k_diag_tiled(Grid g, TArgs<T> args, int ntx, int nty, int ntz,
                                                        T* __restrict__ rho, T* __restrict__ Jd, T* __restrict__ P) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc;
  constexpr int NCELL = TX * TY * TZ;
  constexpr int NPAIR = (NCELL + 1) / 2;
  constexpr int WREC = kDRows * kSlots;
  __shared__ __attribute__((aligned(16))) T smem[NW * WREC + NCELL * kDCell];
  __shared__ TSpecies<T> lsp[kMaxTiledSpecies];
  __shared__ PtrSet<T> lptr_tab[kZeroSlot + 1];
  LdsPtrSet<T>* const lptr = (LdsPtrSet<T>*)lptr_tab;
  T* const scell = smem + NW * WREC;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int half = lane >> 5;
  const int hl = lane & 31;
  const int col = lane & 15;
  const int grp = lane >> 4;
  const int64_t nn = g.nn;
  const T inv_V = T(1.0 / g.V);
  int x0, y0, z0;
  brick_origin<TX, TY, TZ>(ntx, nty, ntz, x0, y0, z0);
  for (int i = tid; i < NW * WREC + NCELL * kDCell; i += NW * 64) smem[i] = T(0);
  fill_tables(args, lsp, lptr_tab, tid);
  __syncthreads();
  T* const wrec = smem + wave * WREC;
  const T* const opnd = wrec + col * kSlots + grp;

  for (int pair = wave; pair < NPAIR; pair += NW) {
    const BrickCell pc = brick_cell<TX, TY, TZ>(g, x0, y0, z0, 2 * pair + half);
    // the cell's list: its species ranges (the stray slot stays empty; its
    // range is not loaded, there being no stray list here)
    const RangeLd rl = load_ranges<T, kMaxTiledSpecies>(args, lsp, pc);
    Ranges rg;
    {
      int e = 0, prev = 0;
#pragma unroll
      for (int s = 0; s < kSlots5; ++s) {
        const bool used = s < args.ns && s != kStraySlot;
        const int dlt = rl.lo[s] - e;
        if (s == 0) rg.d0 = dlt;
        else rg.inc[s - 1] = dlt - prev;
        prev = dlt;
        e += (pc.valid && used) ? rl.hi[s] - rl.lo[s] : 0;
        if (s < kSlots5 - 1) rg.end[s] = e;
      }
      rg.total = e;
    }
    const int cntA = __builtin_amdgcn_readfirstlane(__shfl(rg.total, 0));
    const int cntB = __builtin_amdgcn_readfirstlane(__shfl(rg.total, 32));
    const int cmax = cntA > cntB ? cntA : cntB;
    if (cmax == 0) continue;   // wave-uniform
    acc_t dA = {0, 0, 0, 0}, dB = {0, 0, 0, 0};
    for (int cb = 0; cb < cmax; cb += 32) {
      const PData<T> pd = load_dep<T>(lptr, rg, cb + hl);
      {
        const TSpecies<T>& sp = lsp[dep_species(pd)];
        (void)sp;
        const Stencil<T> ps = particle_stencil<T>(g, pd.x0, pd.x1, pd.x2, pd.c);
        const int pcell = ps.i[0] + g.nx * (ps.i[1] + g.ny * ps.i[2]);
        const bool in_cell = pd.ok && pcell == pc.cell;
        const T q = pd.ok ? dep_charge(pd, lptr) * inv_V : T(0);
        T f[kDVals];
        diag_values(in_cell ? q : T(0), pd.v0, pd.v1, pd.v2, f);
        T W[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) W[a] = corner_weight(ps, a);
#pragma unroll
        for (int i = 0; i < kDVals; ++i) wrec[i * kSlots + lane] = f[i];
#pragma unroll
        for (int a = 0; a < 8; ++a) wrec[(kDVals + a) * kSlots + lane] = W[a];
        if (pd.ok && !in_cell) {   // out of its range's cell: straight to the global arrays
          T fs[kDVals];
          diag_values(q, pd.v0, pd.v1, pd.v2, fs);
#pragma unroll
          for (int a = 0; a < 8; ++a) {
            const int64_t node = corner_node(g, ps, a);
#pragma unroll
            for (int v = 0; v < kDVals; ++v) unsafeAtomicAdd(diag_target(rho, Jd, P, nn, v, node), fs[v] * W[a]);
          }
        }
      }
      wave_sync();
      const int nk = cmax - cb;   // wave-uniform, >= 1
#pragma unroll
      for (int k4 = 0; k4 < 32; k4 += 4) {
        if (k4 > 0 && k4 >= nk) break;
        dA = MF::run(opnd[k4], opnd[kDVals * kSlots + k4], dA);
        dB = MF::run(opnd[32 + k4], opnd[kDVals * kSlots + 32 + k4], dB);
      }
      wave_sync();
    }
    // per-cell sums [value][corner]: rows < 10, columns < 8
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int lch = 2 * pair + h;
      if (lch >= NCELL || col >= 8) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = MF::row(lane, r);
        if (row < kDVals) scell[lch * kDCell + row * 8 + col] = h == 0 ? dA[r] : dB[r];
      }
    }
  }
  __syncthreads();
  // node gather: every (value, node) of the brick sums its <= 8 cells once
  constexpr int NX = TX + 1, NY = TY + 1, NZ = TZ + 1, NN = NX * NY * NZ;
  for (int it = tid; it < kDVals * NN; it += NW * 64) {
    const int v = it / NN, ln = it % NN;
    const int nx_ = ln % NX, ny_ = (ln / NX) % NY, nz_ = ln / (NX * NY);
    T sum = T(0);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int lcx = nx_ - (a & 1), lcy = ny_ - ((a >> 1) & 1), lcz = nz_ - ((a >> 2) & 1);
      if (lcx >= 0 && lcx < TX && lcy >= 0 && lcy < TY && lcz >= 0 && lcz < TZ)
        sum += scell[(lcx + TX * (lcy + TY * lcz)) * kDCell + v * 8 + a];
    }
    const int gx = wrap_once(x0 + nx_, g.nx), gy = wrap_once(y0 + ny_, g.ny), gz = wrap_once(z0 + nz_, g.nz);
    const int64_t gn = gx + (int64_t)g.nx * (gy + (int64_t)g.ny * gz);
    note_nonfinite(g, !finite(sum));
    if (sum != T(0)) unsafeAtomicAdd(diag_target(rho, Jd, P, nn, v, gn), sum);
  }
}

// ---------------------------------------------------------------------------
// stray mover: particles listed before their move -- found outside their
// range's cell -- are moved here with fields read from memory, in the same
// arithmetic as the grouped mover, and their new cell recorded.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_move_strays(Grid g, TArgs<T> args) {
  __shared__ TSpecies<T> lsp[kMaxTiledSpecies];
  __shared__ double red[4];
  fill_tables<T>(args, lsp, nullptr, threadIdx.x);
  __syncthreads();
  const int n = *args.stray_count;
  double kel = 0.0;
  // four entries per thread and pass: their item loads are in flight together
  // (most entries need no move, so the loads set the pace)
  const int stride = gridDim.x * 256;
  for (int i0 = blockIdx.x * 256 + threadIdx.x; i0 < n; i0 += 4 * stride) {
    int items[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) items[e] = i0 + e * stride < n ? args.stray_item[i0 + e * stride] : 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = i0 + e * stride;
      const int item = items[e];
      if (!(item & kUnmoved)) continue;
      const int s = (item >> kItemShift) & (kMaxTiledSpecies - 1);
      const int p = item & kIndexMask;
      const TSpecies<T>& sp = lsp[s];
      const StrayData<T>& ul = args.ul;   // the listed (current) state
      const T q = ul.q[i];
      const T x0 = ul.pos[0][i], x1 = ul.pos[1][i], x2 = ul.pos[2][i];
      Stencil<T> ps = particle_stencil<T>(g, x0, x1, x2, ul.cell[i]);
      T W[8];
      int64_t nd[8];
      corners(g, ps, W, nd);
      const Vec3<T> Ep = gather(args.Emove, g.nn, W, nd);
      const Vec3<T> Bp = gather(args.Bmove, g.nn, W, nd);
      const Vec3<T> v = advance_velocity(Bp, sp.beta, Vec3<T>{ul.vel[0][i], ul.vel[1][i], ul.vel[2][i]}, Ep);
      note_nonfinite(g, !(finite(v.x) && finite(v.y) && finite(v.z)));
      T n0, n1, n2;
      int ncell;
      if constexpr (sizeof(T) == 4) {
        int ix = ps.i[0], iy = ps.i[1], iz = ps.i[2];
        n0 = push_offset(ps.w1[0], v.x, args.dth[0], ix, g.nx);
        n1 = push_offset(ps.w1[1], v.y, args.dth[1], iy, g.ny);
        n2 = push_offset(ps.w1[2], v.z, args.dth[2], iz, g.nz);
        ncell = ix + g.nx * (iy + g.ny * iz);
        gst(sp.cell + p, ncell);
      } else {
        n0 = push_abs(x0, g.pdt[0], v.x, g.nx * g.hx);
        n1 = push_abs(x1, g.pdt[1], v.y, g.ny * g.hy);
        n2 = push_abs(x2, g.pdt[2], v.z, g.nz * g.hz);
        const Stencil<double> nps = stencil_abs(g, n0, n1, n2);
        ncell = nps.i[0] + g.nx * (nps.i[1] + g.ny * nps.i[2]);
      }
      gst(sp.pos[0] + p, n0);
      gst(sp.pos[1] + p, n1);
      gst(sp.pos[2] + p, n2);
      gst(sp.vel[0] + p, v.x);
      gst(sp.vel[1] + p, v.y);
      gst(sp.vel[2] + p, v.z);
      ul.pos[0][i] = n0;
      ul.pos[1][i] = n1;
      ul.pos[2][i] = n2;
      ul.vel[0][i] = v.x;
      ul.vel[1][i] = v.y;
      ul.vel[2][i] = v.z;
      ul.cell[i] = ncell;
      // back in its range's cell: the deposit takes it from the range, so it
      // leaves the list (cell -1)
      const int range_cell = args.stray_cell[i];
      args.stray_cell[i] = ncell == range_cell ? -1 : ncell;
      if (args.stay && ncell == range_cell) atomicAdd(args.stay + (int64_t)s * g.nn + range_cell, 1);
      args.stray_item[i] = item & ~kUnmoved;
      if (args.ke) {
        const double vx = v.x, vy = v.y, vz = v.z;
        kel += 0.5 * ((double)q * sp.inv_qom) * ((vx * vx + vy * vy) + vz * vz);
      }
    }
  }
  if (args.ke) {
    for (int off = 32; off > 0; off >>= 1) kel += __shfl_down(kel, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = kel;
    __syncthreads();
    if (threadIdx.x == 0) {
      const double t = (red[0] + red[1]) + (red[2] + red[3]);
      if (t != 0.0) unsafeAtomicAdd(args.ke, t);
    }
  }
}

// ---------------------------------------------------------------------------
// stray list: rank by cell, then scatter into cell order
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_stray_rank(const int* __restrict__ count, const int* __restrict__ cellv,
                                                    int* __restrict__ counts, int* __restrict__ ranks) {
  // one returning atomic per stray, all lanes at once: strays of a wavefront
  // mostly lie in different cells, so a per-key leader loop would serialise
  // (four entries per thread and pass, their atomics in flight together)
  const int n = *count;
  const int stride = gridDim.x * 256;
  for (int i0 = blockIdx.x * 256 + threadIdx.x; i0 < n; i0 += 4 * stride) {
    int c[4], r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] = i0 + u * stride < n ? cellv[i0 + u * stride] : -1;
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = c[u] >= 0 ? atomicAdd(&counts[c[u]], 1) : 0;   // cell -1: not listed
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (c[u] >= 0) ranks[i0 + u * stride] = r[u];
  }
}

// regrouping: the particles of (species, cell) after the pass, in place of the
// stray counts
// each species' particles per cell after the pass: its stayers plus the
// cell's sorted strays of that species (contiguous from start[c], their
// species stored by the scatter; one thread per cell, no atomics)
__global__ void __launch_bounds__(256) k_regroup_total(int* __restrict__ scount, const int* __restrict__ stay,
                                                       const int* __restrict__ start, const int32_t* __restrict__ ssp,
                                                       int ns, int64_t nn) {
  for (int64_t c = blockIdx.x * 256 + threadIdx.x; c < nn; c += (int64_t)gridDim.x * 256) {
    int cnt[kMaxTiledSpecies] = {0, 0, 0, 0};
    const int e = start[c + 1];
    for (int i = start[c]; i < e; ++i) {
      const int sp = ssp[i];
#pragma unroll
      for (int k = 0; k < kMaxTiledSpecies; ++k) cnt[k] += sp == k ? 1 : 0;
    }
#pragma unroll
    for (int k = 0; k < kMaxTiledSpecies; ++k)
      if (k < ns) scount[k * nn + c] = stay[k * nn + c] + cnt[k];
  }
}

// regrouping: the cell ranges of each species from the scan over (species, cell)
template <typename T>
__global__ void __launch_bounds__(256) k_regroup_starts(TArgs<T> args, const int* __restrict__ scan, int64_t nn) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < (int64_t)args.ns * (nn + 1); i += (int64_t)gridDim.x * 256) {
    const int s = (int)(i / (nn + 1));
    const int64_t c = i % (nn + 1);
    args.dst[s].start[c] = scan[s * nn + c] - scan[s * nn];
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_stray_scatter(TArgs<T> args, const int* __restrict__ ranks) {
  // two entries per thread and pass, their loads in flight together
  const int n = *args.stray_count;
  const int stride = gridDim.x * 256;
  const StrayData<T>& u = args.ul;
  const StrayData<T>& d = args.sd;
  for (int i0 = blockIdx.x * 256 + threadIdx.x; i0 < n; i0 += 2 * stride) {
    int c[2], o[2], sp[2], cl[2];
    T v[2][7];
#pragma unroll
    for (int h = 0; h < 2; ++h) c[h] = i0 + h * stride < n ? args.stray_cell[i0 + h * stride] : -1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = c[h] >= 0 ? i0 + h * stride : 0;
      const int cc = c[h] >= 0 ? c[h] : 0;
      o[h] = args.ind_start[cc] + ranks[i];
      for (int k = 0; k < 3; ++k) {
        v[h][k] = u.pos[k][i];
        v[h][3 + k] = u.vel[k][i];
      }
      v[h][6] = u.q[i];
      cl[h] = u.cell[i];
      sp[h] = (args.stray_item[i] >> kItemShift) & (kMaxTiledSpecies - 1);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (c[h] < 0) continue;
      for (int k = 0; k < 3; ++k) {
        d.pos[k][o[h]] = v[h][k];
        d.vel[k][o[h]] = v[h][3 + k];
      }
      d.q[o[h]] = v[h][6];
      d.cell[o[h]] = cl[h];
      d.sp[o[h]] = sp[h];
    }
  }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace of the tiled path: the stray counter, a zero block and a sink
// (256 bytes each),
// the stray list (item, cell, rank), the strays' state in list order (7
// arrays of esz-byte values and the cell) and in cell order (the same and the
// species), the per-cell stray counts and their scan. Laid out by carve();
// tiled_workspace_bytes() is its size.
struct StrayWs {
  int* count;
  void* zero;
  void* sink;
  int* item;
  int* cell;
  int* rank;
  void* udata[7];  // listed state in list order: pos[3], vel[3], q
  int* ucell;
  void* data[7];   // ... and in cell order
  int* dcell;
  int* dsp;
  int* counts;
  int* start;
  int* scan_sums;
  int* stay;       // regrouping: [species][cell] stayers, strays (then totals), their scan
  int* scount;
  int* rscan;
  int* rsums;
  void* csum;      // per-cell sums of the deposit, [cells][SCS]
};


StrayWs carve(const Grid& g, int64_t cap, size_t esz, void* ws) {
  // the per-cell sums first: [cells][SCS] values
  char* w0 = (char*)ws;
  void* csum = w0;
  ws = w0 + align256(esz * SCS * (size_t)g.nn);
  char* w = (char*)ws;
  StrayWs s;
  // the counter (hit by atomics), the zero block (read by every idle or
  // constant-charge lane) and the sink (written by idle lanes) on cache
  // lines of their own
  s.count = (int*)w;
  s.zero = w + 256;
  s.sink = w + 512;
  w += 768;
  s.item = (int*)w;
  w += align256(sizeof(int) * (size_t)cap);
  s.cell = (int*)w;
  w += align256(sizeof(int) * (size_t)cap);
  s.rank = (int*)w;
  w += align256(sizeof(int) * (size_t)cap);
  for (int k = 0; k < 7; ++k) {
    s.udata[k] = w;
    w += align256(esz * (size_t)cap);
  }
  s.ucell = (int*)w;
  w += align256(sizeof(int) * (size_t)cap);
  for (int k = 0; k < 7; ++k) {
    s.data[k] = w;
    w += align256(esz * (size_t)cap);
  }
  s.dcell = (int*)w;
  w += align256(sizeof(int) * (size_t)cap);
  s.dsp = (int*)w;
  w += align256(sizeof(int) * (size_t)cap);
  s.counts = (int*)w;
  w += align256(sizeof(int) * (size_t)g.nn);
  s.start = (int*)w;
  w += align256(sizeof(int) * (size_t)(g.nn + 1));
  s.scan_sums = (int*)w;
  w += align256(sizeof(int) * (size_t)scan_sums_ints(g.nn));
  s.stay = (int*)w;
  w += align256(sizeof(int) * kMaxTiledSpecies * (size_t)g.nn);
  s.scount = (int*)w;
  w += align256(sizeof(int) * kMaxTiledSpecies * (size_t)g.nn);
  s.rscan = (int*)w;
  w += align256(sizeof(int) * (kMaxTiledSpecies * (size_t)g.nn + 1));
  s.rsums = (int*)w;
  s.csum = csum;
  return s;
}

template <typename T>
TArgs<T> make_args(const Grid& g, const SpeciesArgs* sp, int ns) {
  TArgs<T> a{};
  a.ns = ns;
  for (int s = 0; s < ns; ++s) {
    for (int d = 0; d < 3; ++d) {
      a.s[s].pos[d] = (T*)sp[s].pos[d];
      a.s[s].vel[d] = (T*)sp[s].vel[d];
    }
    a.s[s].cell = sp[s].cell;
    a.s[s].q = (const T*)sp[s].q;
    a.s[s].q_const = (T)sp[s].q_const;
    a.s[s].beta = (T)(sp[s].qom * g.dt / 2.0);
    a.s[s].beta_V = (T)(sp[s].qom * g.dt / 2.0 / g.V);
    a.s[s].inv_V = (T)(1.0 / g.V);
    a.s[s].inv_qom = 1.0 / integrated_qom(sp[s].qom, g.dt, sizeof(T) == 4);
    a.s[s].cell_start = sp[s].cell_start;
    a.s[s].np = sp[s].np;
  }
  a.dth[0] = (T)(g.pdt[0] / g.hx);
  a.dth[1] = (T)(g.pdt[1] / g.hy);
  a.dth[2] = (T)(g.pdt[2] / g.hz);
  return a;
}

// grouped pass (move or check) -> [stray mover] -> stray counting sort -> deposit
template <typename T, int TX, int TY, int TZ, int NW>
hipError_t run_T(const Grid& g, const SpeciesArgs* sp, int ns, const void* Emove, const void* Bmove,
                 const void* Bdep, void* J, void* M, double* ke, bool move, bool accumulate, void* ws,
                 hipStream_t st, const SpeciesArgs* dst = nullptr) {
  const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + TZ - 1) / TZ;
  const int ntiles = ntx * nty * ntz;
  int64_t cap = 0;
  for (int s = 0; s < ns; ++s) cap += sp[s].np;
  StrayWs w = carve(g, cap, sizeof(T), ws);
  hipError_t e = launch_zero(w.count, 512, st);   // the counter and the zero block
  if (e != hipSuccess) return e;
  TArgs<T> a = make_args<T>(g, sp, ns);
  a.Bdep = (const T*)Bdep;
  a.Emove = (const T*)Emove;
  a.Bmove = (const T*)Bmove;
  a.stray_count = w.count;
  a.stray_item = w.item;
  a.stray_cell = w.cell;
  a.ke = ke;
  a.csum = (T*)w.csum;
  a.zero = w.zero;
  a.sink = w.sink;
  a.ind_start = w.start;
  for (int k = 0; k < 3; ++k) {
    a.sd.pos[k] = (T*)w.data[k];
    a.sd.vel[k] = (T*)w.data[3 + k];
  }
  a.sd.q = (T*)w.data[6];
  a.sd.cell = w.dcell;
  a.sd.sp = w.dsp;
  for (int k = 0; k < 3; ++k) {
    a.ul.pos[k] = (T*)w.udata[k];
    a.ul.vel[k] = (T*)w.udata[3 + k];
  }
  a.ul.q = (T*)w.udata[6];
  a.ul.cell = w.ucell;
  a.ul.sp = nullptr;
  const bool regroup = dst != nullptr;
  if (regroup) {
    a.stay = w.stay;
    a.scount = w.scount;
    for (int s = 0; s < ns; ++s) {
      for (int d = 0; d < 3; ++d) {
        a.dst[s].pos[d] = (T*)dst[s].pos[d];
        a.dst[s].vel[d] = (T*)dst[s].vel[d];
      }
      a.dst[s].q = (T*)dst[s].q;
      a.dst[s].cell = dst[s].cell;
      a.dst[s].start = const_cast<int32_t*>(dst[s].cell_start);
      a.dst[s].np = dst[s].np;
    }
  }
  constexpr int kGroupWaves = 4;   // 4-wave workgroups: three fit a CU at the mover's register count
  if (move) {
    hipLaunchKernelGGL((k_mover<T, TX, TY, TZ, kGroupWaves>), dim3(ntiles), dim3(kGroupWaves * 64), 0, st, g, a, ntx,
                       nty, ntz);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_move_strays<T>, dim3(1024), dim3(256), 0, st, g, a);
  } else {
    hipLaunchKernelGGL((k_group<T, TX, TY, TZ, kGroupWaves, false>), dim3(ntiles), dim3(kGroupWaves * 64), 0, st, g,
                       a, ntx, nty, ntz);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // strays: counting sort by cell
  if ((e = launch_zero(w.counts, sizeof(int) * (size_t)g.nn, st)) != hipSuccess) return e;
  const int64_t nsn = (int64_t)ns * g.nn;
  hipLaunchKernelGGL(k_stray_rank, dim3(1024), dim3(256), 0, st, (const int*)w.count, (const int*)w.cell, w.counts,
                     w.rank);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_exclusive_scan(w.counts, g.nn, w.start, w.scan_sums, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_stray_scatter<T>, dim3(1024), dim3(256), 0, st, a, (const int*)w.rank);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (regroup) {
    // the species' cell ranges after the pass: stayers plus arriving strays
    hipLaunchKernelGGL(k_regroup_total, dim3(1024), dim3(256), 0, st, w.scount, (const int*)w.stay,
                       (const int*)w.start, (const int32_t*)w.dsp, ns, g.nn);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_exclusive_scan(w.scount, nsn, w.rscan, w.rsums, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_regroup_starts<T>, dim3(1024), dim3(256), 0, st, a, (const int*)w.rscan, g.nn);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_deposit<T, TX, TY, TZ, NW, true>), dim3(ntiles), dim3(NW * 64), 0, st, g, a, ntx, nty,
                       ntz);
  } else {
    hipLaunchKernelGGL((k_deposit<T, TX, TY, TZ, NW, false>), dim3(ntiles), dim3(NW * 64), 0, st, g, a, ntx, nty,
                       ntz);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // node bricks of the flush, one workgroup of 1024 threads per CU (16
  // wavefronts of staging loads in flight): FP32 8 x 4 x 2 (135 staged
  // cells, 142 KB of LDS, each record read 2.1 times instead of 2.3 with
  // 4 x 4 x 2 bricks), measured 128 us against 154 with 4 x 4 x 2 bricks
  // of 256 threads at 64^3; FP64 4 x 4 x 2 (75 cells, 158 KB), 261 us
  // against 379 with 4 x 2 x 2 bricks of 256 threads
  constexpr int FX = sizeof(T) == 4 ? 8 : 4, FY = 4, FZ = 2;
  const int nbx = (g.nx + FX - 1) / FX, nby = (g.ny + FY - 1) / FY, nbz = (g.nz + FZ - 1) / FZ;
  constexpr int NT = 1024;
  hipLaunchKernelGGL((k_flush_nodes<T, FX, FY, FZ, NT>), dim3((unsigned)(nbx * nby * nbz)), dim3(NT), 0, st, g,
                     (const T*)w.csum, (T*)J, (T*)M, accumulate ? 1 : 0, nbx, nby, nbz);
  return hipGetLastError();
}

}  // namespace

namespace {
template <typename T, int TX, int TY, int TZ, int NW>
hipError_t run_diag(const Grid& g, const SpeciesArgs* sp, int ns, void* rho, void* Jd, void* P, void* zero,
                    hipStream_t st) {
  const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + TZ - 1) / TZ;
  TArgs<T> a = make_args<T>(g, sp, ns);
  a.zero = zero;
  hipError_t e = launch_zero(zero, 256, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_diag_tiled<T, TX, TY, TZ, NW>), dim3(ntx * nty * ntz), dim3(NW * 64), 0, st, g, a, ntx, nty,
                     ntz, (T*)rho, (T*)Jd, (T*)P);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_diagnostics_tiled(const Grid& g, bool f32, const SpeciesArgs* sp, int ns, void* rho, void* Jd,
                                    void* P, void* zero, hipStream_t st) {
  if (g.nz == 1) {
    if (f32) return run_diag<float, 8, 4, 1, 4>(g, sp, ns, rho, Jd, P, zero, st);
    return run_diag<double, 8, 4, 1, 4>(g, sp, ns, rho, Jd, P, zero, st);
  }
  if (f32) return run_diag<float, 4, 4, 2, 4>(g, sp, ns, rho, Jd, P, zero, st);
  return run_diag<double, 4, 4, 2, 4>(g, sp, ns, rho, Jd, P, zero, st);
}

size_t tiled_workspace_bytes(const Grid& g, int64_t np_total, bool f32) {
  const size_t esz = f32 ? 4 : 8;
  return align256(esz * SCS * (size_t)g.nn) + 768 + 6 * align256(sizeof(int) * (size_t)np_total) + 14 * align256(esz * (size_t)np_total) +
         align256(sizeof(int) * (size_t)g.nn) + align256(sizeof(int) * (size_t)(g.nn + 1)) +
         align256(sizeof(int) * (size_t)scan_sums_ints(g.nn)) +
         2 * align256(sizeof(int) * kMaxTiledSpecies * (size_t)g.nn) +
         align256(sizeof(int) * (kMaxTiledSpecies * (size_t)g.nn + 1)) +
         sizeof(int) * (size_t)scan_sums_ints(kMaxTiledSpecies * g.nn);
}

bool tiled_species_ok(const SpeciesArgs* sp, int ns) {
  if (ns > kMaxTiledSpecies) return false;
  for (int s = 0; s < ns; ++s)
    if (sp[s].np >= (1 << kItemShift)) return false;
  return true;
}

hipError_t launch_deposit_tiled(const Grid& g, bool f32, const SpeciesArgs* sp, int ns, const void* B, void* J,
                                void* M, bool accumulate, void* ws, hipStream_t st) {
  // single-layer (2D) grids take 8x4x1 bricks, so that no brick cell is empty
  if (g.nz == 1) {
    if (f32) return run_T<float, 8, 4, 1, 4>(g, sp, ns, nullptr, nullptr, B, J, M, nullptr, false, accumulate, ws, st);
    return run_T<double, 8, 4, 1, 2>(g, sp, ns, nullptr, nullptr, B, J, M, nullptr, false, accumulate, ws, st);
  }
  if (f32) return run_T<float, 4, 4, 2, 4>(g, sp, ns, nullptr, nullptr, B, J, M, nullptr, false, accumulate, ws, st);
  return run_T<double, 4, 4, 2, 2>(g, sp, ns, nullptr, nullptr, B, J, M, nullptr, false, accumulate, ws, st);
}

hipError_t launch_move_deposit_regroup(const Grid& g, bool f32, const SpeciesArgs* sp, const SpeciesArgs* dst, int ns,
                                       const void* E, const void* B, const void* Bnext, void* J, void* M, double* ke,
                                       bool accumulate, void* ws, hipStream_t st) {
  if (g.nz == 1) {
    if (f32) return run_T<float, 8, 4, 1, 4>(g, sp, ns, E, B, Bnext, J, M, ke, true, accumulate, ws, st, dst);
    return run_T<double, 8, 4, 1, 2>(g, sp, ns, E, B, Bnext, J, M, ke, true, accumulate, ws, st, dst);
  }
  if (f32) return run_T<float, 4, 4, 2, 4>(g, sp, ns, E, B, Bnext, J, M, ke, true, accumulate, ws, st, dst);
  return run_T<double, 4, 4, 2, 2>(g, sp, ns, E, B, Bnext, J, M, ke, true, accumulate, ws, st, dst);
}

hipError_t launch_move_deposit(const Grid& g, bool f32, const SpeciesArgs* sp, int ns, const void* E, const void* B,
                               const void* Bnext, void* J, void* M, double* ke, bool accumulate, void* ws,
                               hipStream_t st) {
  if (g.nz == 1) {
    if (f32) return run_T<float, 8, 4, 1, 4>(g, sp, ns, E, B, Bnext, J, M, ke, true, accumulate, ws, st);
    return run_T<double, 8, 4, 1, 2>(g, sp, ns, E, B, Bnext, J, M, ke, true, accumulate, ws, st);
  }
  if (f32) return run_T<float, 4, 4, 2, 4>(g, sp, ns, E, B, Bnext, J, M, ke, true, accumulate, ws, st);
  return run_T<double, 4, 4, 2, 2>(g, sp, ns, E, B, Bnext, J, M, ke, true, accumulate, ws, st);
}

}  // namespace ecsim
