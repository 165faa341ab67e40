// Host-side declarations shared by the C-ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "device.h"

namespace ecsim {

// A species as the launchers see it (validated by the C-ABI layer).
struct SpeciesArgs {
  int np;
  double qom;
  void* pos[3];
  int32_t* cell;
  void* vel[3];
  const void* q;
  double q_const;
  const int32_t* cell_start;
};

constexpr int kMaxSpecies = 8;

// The kernels carry beta = (q/m) dt / 2 of a species as a constant in the
// particles' precision, so they move particles whose charge-to-mass ratio is
// 2 beta / dt (in FP32 that differs from q/m by the rounding of beta, 1.5e-8
// relative for q/m = -1, dt = 0.1). The scheme exchanges energy exactly
// between the fields and those particles (Secs. I-II), so the kinetic energy
// takes their masses, q_p dt / (2 beta).
inline double integrated_qom(double qom, double dt, bool f32) {
  const double beta = qom * dt / 2.0;
  return 2.0 * (f32 ? (double)(float)beta : beta) / dt;
}

hipError_t launch_move(const Grid& g, bool f32, const SpeciesArgs& sp, const void* E, const void* B,
                       double* ke, hipStream_t st);

hipError_t launch_diagnostics_atomic(const Grid& g, bool f32, const SpeciesArgs* sp, int ns, void* rho, void* Jd,
                                     void* P, void* acc, hipStream_t st);
hipError_t launch_diagnostics_tiled(const Grid& g, bool f32, const SpeciesArgs* sp, int ns, void* rho, void* Jd,
                                    void* P, void* zero, hipStream_t st);
hipError_t launch_deposit_atomic(const Grid& g, bool f32, const SpeciesArgs* sp, int ns, const void* B,
                                 void* J, void* M, hipStream_t st);

// Tiled deposit over particles grouped by cell ranges (cell_start); particles
// outside their range's cell are handled through a stray list in `ws`.
size_t tiled_workspace_bytes(const Grid& g, int64_t np_total, bool f32);
bool tiled_species_ok(const SpeciesArgs* sp, int ns);
// J and M are written (accumulate: added to) by the node flush; they need
// no clearing.
hipError_t launch_deposit_tiled(const Grid& g, bool f32, const SpeciesArgs* sp, int ns, const void* B,
                                void* J, void* M, bool accumulate, void* ws, hipStream_t st);
// Fused mover + deposit: moves every species with (E, B) and deposits the
// moments at the new positions with Bnext.
hipError_t launch_move_deposit(const Grid& g, bool f32, const SpeciesArgs* sp, int ns, const void* E,
                               const void* B, const void* Bnext, void* J, void* M, double* ke, bool accumulate,
                               void* ws, hipStream_t st);
// Fused mover + deposit that also regroups: each species' particles are
// written to dst[s] in cell order (the deposit's order) and dst[s].cell_start
// receives the ranges.
hipError_t launch_move_deposit_regroup(const Grid& g, bool f32, const SpeciesArgs* sp, const SpeciesArgs* dst, int ns,
                                       const void* E, const void* B, const void* Bnext, void* J, void* M, double* ke,
                                       bool accumulate, void* ws, hipStream_t st);
// exclusive scan of n < 2^31 ints into out[0..n], out[n] = total; sums:
// scratch of scan_sums_ints(n) ints
int64_t scan_sums_ints(int64_t n);
hipError_t launch_exclusive_scan(const int* in, int64_t n, int* out, int* sums, hipStream_t st);

size_t sort_workspace_bytes(const Grid& g, int64_t np);
hipError_t launch_sort(const Grid& g, bool f32, const SpeciesArgs& src, const SpeciesArgs& dst,
                       int32_t* cell_start, int32_t* perm, void* ws, hipStream_t st);

hipError_t launch_mass_apply(const Grid& g, bool f32, const void* M, const double* x, double a, double b,
                             double* y, hipStream_t st);
hipError_t launch_centres_to_nodes(const Grid& g, const double* BC, double* BN, float* BN32, hipStream_t st);
hipError_t launch_to_f32(int64_t n, const double* src, float* dst, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
// *out = *flag, then *flag = 0 (one thread, on the stream)
hipError_t launch_take_flag(int* flag, int32_t* out, hipStream_t st);

// Field solve (FP64 GMRES). Every kernel takes one node per thread in
// workgroups of kSolveBlock threads and writes or reads per-workgroup
// partial sums over solve_blocks(g) slots.
constexpr int kSolveBlock = 1024;
constexpr int kMaxRestart = 120;
constexpr int kDotBlocks = 256;  // partials of launch_sumsq
int solve_blocks(const Grid& g);
// (c theta dt)^2 / (16 h_r h_c): the run-time factors of the curl-curl
// stencil, whose integer weights the operator kernels hold as constants
struct CurlK {
  double k[3][3];
};
void curl_curl_stencil(const Grid& g, double ctd2, CurlK& K);
// Device state of the Arnoldi process. rb: [0] convergence threshold,
// [1] |r| at the cycle's start, [4, 4 + m) hist, then four ints (active,
// columns that count, columns of the update in X, columns of yn); Pb: the
// partial sums of |b|^2.
struct GmresState {
  double* H;   // (m + 1) x m
  double* cs;  // m
  double* sn;  // m
  double* gv;  // m + 1
  double* h1;  // first Gram-Schmidt pass, m
  double* h2;  // second pass, m
  double* yn;  // least-squares solution over the columns so far, m
  double* yp;  // the one the iterate holds, m
  double* rb;
  const double* Pb;
  int m;
  double tol;
};
enum { kArnoldiNone = 0, kArnoldiStart = 1, kArnoldiGivens = 2 };
// R = b - A E^n with b = E^n + c_j J + c_b curl_N B_C formed on the way
// (E_t = E^n); Pb, Pr: partial |b|^2 and |R|^2 (Pr = Pb + solve_blocks(g))
hipError_t launch_residual_first(const Grid& g, bool mf32, const void* M, const CurlK& K, double cm,
                                 const double* E_n, const void* J, const double* BC, double c_j, double c_b,
                                 double* b, double* E_t, double* R, double* Pb, double* Pr, hipStream_t st);
// R = b - A E_t, Pr: partial |R|^2, the field advance from E_t, and yp = yn
hipError_t launch_residual_last(const Grid& g, bool mf32, const void* M, const CurlK& K, double cm,
                                const double* E_t, const double* b, double* R, double* Pr, const double* E_n,
                                const double* BC_n, double ctd, double* E_next, double* BC_next,
                                const GmresState& G, hipStream_t st);
// step s: V_s = Win / |Win| (|Win|^2 from P3), Wout = A V_s, P1: partial
// <V_v, Wout>, v <= s; mode: start the cycle or close column s - 1
hipError_t launch_arnoldi_op(const Grid& g, bool mf32, const void* M, const CurlK& K, double cm,
                             const double* Win, double* Wout, double* V, int64_t ld, int s, int mode,
                             const double* P3, double* P1, const GmresState& G, hipStream_t st);
// W -= sum_{v<k} h_v V_v with h from the partials Pin (stored to coef);
// Pout: the partials <V_v, W> (norm false) or |W|^2 (norm true)
hipError_t launch_cgs_pass(const Grid& g, bool norm, const double* V, int64_t ld, int k, const double* Pin,
                           double* coef, double* W, double* Pout, hipStream_t st);
// Givens update of column j and y over the columns so far (one workgroup)
hipError_t launch_givens_tail(const Grid& g, int j, const double* P3, const GmresState& G, hipStream_t st);
// X += V (yn - yp)
hipError_t launch_update_x(const Grid& g, const double* V, int64_t ld, double* X, const GmresState& G,
                           hipStream_t st);
// E^{n+1}, B^{n+1} from E^{n+theta}; with G, also yp = yn
hipError_t launch_finish(const Grid& g, const double* E_n, const double* E_t, const double* BC_n, double ctd,
                         double* E_next, double* BC_next, const GmresState* G, hipStream_t st);
hipError_t launch_sumsq(const double* x, int64_t n, double scale, double* partial, double* out, bool accumulate,
                        hipStream_t st);

// Adjoint of (mover ->) moments of one species. With sp.cell_start the
// brick-tiled kernel runs, and ws (backward_workspace_bytes) holds the list of
// particles it leaves to the list kernel and every cell's table; without it
// one thread per particle reads every grid value from memory.
size_t backward_workspace_bytes(const Grid& g, int64_t np, bool f32);
hipError_t launch_backward(const Grid& g, bool f32, const SpeciesArgs& sp, const void* E, const void* B,
                           const void* gJ, const void* gM, void* const gpos[3], void* const gvel[3], void* gE,
                           void* gB, bool through_mover, bool offset_grad, void* ws, hipStream_t st);

}  // namespace ecsim
