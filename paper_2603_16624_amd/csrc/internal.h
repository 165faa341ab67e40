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

// field-solve building blocks (FP64)
hipError_t launch_curl_C(const Grid& g, const double* E, double* out, hipStream_t st);
hipError_t launch_field_op_curl(const Grid& g, const double* E, const double* curlC_E, double ctd2,
                                double* out, hipStream_t st);
hipError_t launch_rhs(const Grid& g, const double* E_n, bool jf32, const void* J, const double* BC, double c_j,
                      double c_b, double* b, hipStream_t st);
hipError_t launch_finish(const Grid& g, const double* E_n, const double* E_t, const double* BC_n,
                         const double* curlC_Et, double ctd, double* E_next, double* BC_next, hipStream_t st);
// out[v] = <V_v, w> for v < nv (V_v = V + v*ld); partial: >= nv*kDotBlocks doubles
constexpr int kDotBlocks = 256;
hipError_t launch_dots(const double* V, int64_t ld, int nv, const double* w, int64_t n, double* partial,
                       double* out, hipStream_t st);
// w -= sum_v coef[v] V_v  (coef: host array of nv <= kMaxRestart + 1 values,
// passed to the kernel by value)
constexpr int kMaxRestart = 120;
hipError_t launch_sub_combo(const double* V, int64_t ld, int nv, const double* coef_host, double* w, int64_t n,
                            hipStream_t st);
// w -= sum_v coef[v] V_v with device coefficients
hipError_t launch_sub_combo_dev(const double* V, int64_t ld, int nv, const double* coef_dev, double* w, int64_t n,
                                hipStream_t st);
// out = w / sqrt(*nrm2)
hipError_t launch_normalize(const double* w, const double* nrm2, double* out, int64_t n, hipStream_t st);
// the device-side GMRES bookkeeping: one Arnoldi column with its Givens
// rotation, the start of a restart cycle, the final back substitution
hipError_t launch_givens(int j, int m, double* H, double* cs, double* sn, double* gv, const double* h1,
                         const double* h2, const double* hn2, double thresh, int* state, double* hist,
                         hipStream_t st);
hipError_t launch_gmres_start(int m, double beta, double* gv, int* state, hipStream_t st);
hipError_t launch_backsolve(const double* H, const double* gv, int m, int j, double* ny, hipStream_t st);
// y = a x + b y
hipError_t launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st);
hipError_t launch_scale_copy(int64_t n, double a, const double* x, double* y, hipStream_t st);
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
