// C ABI of the ECsim hot path: argument validation, dispatch to the kernel
// launchers on the caller's stream, and the host driver of the FP64 GMRES
// field solve (Eqs. 6-7). Declarations and the contract of every entry point
// are in include/ecsim.h.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/ecsim.h"
#include "internal.h"

using namespace ecsim;

namespace {

thread_local char g_err[512] = "no error";

ecsim_status fail(ecsim_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

ecsim_status hip_fail(hipError_t e, const char* where) {
  return fail(ECSIM_EHIP, "%s: %s", where, hipGetErrorString(e));
}

constexpr double kPi = 3.14159265358979323846;
constexpr double kTheta = 0.5;
constexpr double kC = 1.0;

// The per-device record of non-finite values: kernels of the mover, the
// moment deposits and the adjoint set it when they produce a value that is not
// finite; ecsim_check_finite / ecsim_nonfinite_read report and clear it. Every
// device that runs the library holds its own copy, whose address is looked up
// once per device.
__device__ __attribute__((aligned(256))) int g_nonfinite[64];

constexpr int kMaxDevices = 64;
std::mutex g_flag_mu;
int* g_flag_ptr[kMaxDevices] = {};

int* device_flag() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_flag_mu);
  if (!g_flag_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_nonfinite)) != hipSuccess || !p) return nullptr;
    g_flag_ptr[dev] = (int*)p;
  }
  return g_flag_ptr[dev];
}

// Scratch of ecsim_move_moments_noalloc, in place of a caller's workspace: a
// file-scope device array, which every device that runs the library holds
// (its own copy, at its own address) until the process ends. Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol): the device address of the current device's copy is looked up
// once per device and kept.
__device__ __attribute__((aligned(256))) unsigned char scratch[ECSIM_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* device_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

// Attaches the current device's non-finite flag to a validated grid, right
// before the first launch of an entry point.
ecsim_status bind_flag(Grid& g, const char* who) {
  g.nonfinite = device_flag();
  if (!g.nonfinite) return fail(ECSIM_EHIP, "%s: the device's non-finite flag is not accessible", who);
  return ECSIM_OK;
}

ecsim_status make_grid(const ecsim_grid* gr, Grid& g) {
  if (!gr) return fail(ECSIM_EINVAL, "grid is NULL");
  for (int d = 0; d < 3; ++d) {
    if (gr->n[d] < 1) return fail(ECSIM_EINVAL, "grid n[%d] = %d must be >= 1", d, gr->n[d]);
    if (!(gr->h[d] > 0.0) || !std::isfinite(gr->h[d])) return fail(ECSIM_EINVAL, "grid h[%d] must be > 0", d);
  }
  if (!(gr->dt > 0.0) || !std::isfinite(gr->dt)) return fail(ECSIM_EINVAL, "grid dt must be > 0");
  int64_t nn = (int64_t)gr->n[0] * gr->n[1] * gr->n[2];
  if (nn >= ((int64_t)1 << 31)) return fail(ECSIM_EINVAL, "grid has %lld cells; at most 2^31 - 1", (long long)nn);
  g.nx = gr->n[0];
  g.ny = gr->n[1];
  g.nz = gr->n[2];
  g.hx = gr->h[0];
  g.hy = gr->h[1];
  g.hz = gr->h[2];
  g.dt = gr->dt;
  g.nn = nn;
  g.V = gr->h[0] * gr->h[1] * gr->h[2];
  // the mover's fixPosition step for reduced (1D/2D) runs: no push along a
  // dimension of a single cell
  for (int d = 0; d < 3; ++d) g.pdt[d] = gr->n[d] > 1 ? gr->dt : 0.0;
  g.nonfinite = nullptr;
  g.div_x = make_fastdiv((uint32_t)g.nx);
  g.div_xy = make_fastdiv((uint32_t)((int64_t)g.nx * g.ny));
  return ECSIM_OK;
}

ecsim_status check_prec(int32_t prec) {
  if (prec != ECSIM_F64 && prec != ECSIM_F32) return fail(ECSIM_EINVAL, "precision %d is not ECSIM_F64/ECSIM_F32", prec);
  return ECSIM_OK;
}

ecsim_status make_species(const ecsim_particles* sp, SpeciesArgs& a, const char* name) {
  if (!sp) return fail(ECSIM_EINVAL, "%s: particles pointer is NULL", name);
  if (check_prec(sp->prec) != ECSIM_OK) return ECSIM_EINVAL;
  if (sp->np < 0 || sp->np >= ((int64_t)1 << 31)) return fail(ECSIM_EINVAL, "%s: np = %lld out of range", name, (long long)sp->np);
  if (!std::isfinite(sp->qom) || sp->qom == 0.0) return fail(ECSIM_EINVAL, "%s: qom must be finite and non-zero", name);
  if (sp->np > 0) {
    for (int d = 0; d < 3; ++d)
      if (!sp->pos[d] || !sp->vel[d]) return fail(ECSIM_EINVAL, "%s: position/velocity pointer %d is NULL", name, d);
    if (sp->prec == ECSIM_F32 && !sp->cell) return fail(ECSIM_EINVAL, "%s: FP32 particles need a cell array", name);
  }
  if (sp->prec == ECSIM_F64 && sp->cell) return fail(ECSIM_EINVAL, "%s: FP64 particles take no cell array", name);
  if (!sp->q && !std::isfinite(sp->q_const)) return fail(ECSIM_EINVAL, "%s: q_const must be finite", name);
  a.np = (int)sp->np;
  a.qom = sp->qom;
  for (int d = 0; d < 3; ++d) {
    a.pos[d] = sp->pos[d];
    a.vel[d] = sp->vel[d];
  }
  a.cell = sp->cell;
  a.q = sp->q;
  a.q_const = sp->q_const;
  a.cell_start = sp->cell_start;
  return ECSIM_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

const char* ecsim_last_error(void) { return g_err; }

const char* ecsim_version(void) { return "ecsim-mi355x 0.1 (gfx950)"; }

ecsim_status ecsim_workspace_size(const ecsim_grid* grid, int64_t np, int32_t prec, uint32_t flags, size_t* bytes) {
  (void)flags;
  Grid g;
  if (make_grid(grid, g) != ECSIM_OK) return ECSIM_EINVAL;
  if (check_prec(prec) != ECSIM_OK) return ECSIM_EINVAL;
  if (!bytes) return fail(ECSIM_EINVAL, "bytes is NULL");
  if (np < 0 || np >= ((int64_t)1 << 31)) return fail(ECSIM_EINVAL, "np out of range");
  const size_t a = sort_workspace_bytes(g, np), b = tiled_workspace_bytes(g, np, prec == ECSIM_F32);
  *bytes = a > b ? a : b;
  return ECSIM_OK;
}

ecsim_status ecsim_species_qom(int32_t prec, double qom, double dt, double* out) {
  if (check_prec(prec) != ECSIM_OK) return ECSIM_EINVAL;
  if (!out) return fail(ECSIM_EINVAL, "ecsim_species_qom: out is NULL");
  if (!std::isfinite(qom) || qom == 0.0) return fail(ECSIM_EINVAL, "ecsim_species_qom: qom must be finite and non-zero");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ECSIM_EINVAL, "ecsim_species_qom: dt must be > 0");
  *out = integrated_qom(qom, dt, prec == ECSIM_F32);
  return ECSIM_OK;
}

ecsim_status ecsim_move(const ecsim_grid* grid, const ecsim_particles* sp, const void* E_node, const void* B_node,
                        double* ke_out, void* stream) {
  Grid g;
  SpeciesArgs a;
  if (make_grid(grid, g) != ECSIM_OK) return ECSIM_EINVAL;
  if (make_species(sp, a, "ecsim_move") != ECSIM_OK) return ECSIM_EINVAL;
  if (!E_node || !B_node) return fail(ECSIM_EINVAL, "ecsim_move: E_node and B_node are required");
  if (bind_flag(g, "ecsim_move") != ECSIM_OK) return ECSIM_EHIP;
  hipError_t e = launch_move(g, sp->prec == ECSIM_F32, a, E_node, B_node, ke_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ecsim_move");
  return ECSIM_OK;
}

namespace {

ecsim_status species_list(const ecsim_grid* grid, const ecsim_particles* species, int32_t nspecies, Grid& g,
                          SpeciesArgs* a, const char* who, uint32_t flags, bool need_sorted) {
  if (make_grid(grid, g) != ECSIM_OK) return ECSIM_EINVAL;
  if (nspecies < 1 || nspecies > kMaxSpecies)
    return fail(ECSIM_EINVAL, "%s: nspecies = %d not in 1..%d", who, nspecies, kMaxSpecies);
  if (!species) return fail(ECSIM_EINVAL, "%s: species is NULL", who);
  const int32_t prec = species[0].prec;
  for (int s = 0; s < nspecies; ++s) {
    if (make_species(&species[s], a[s], who) != ECSIM_OK) return ECSIM_EINVAL;
    if (species[s].prec != prec) return fail(ECSIM_EINVAL, "%s: species have mixed precisions", who);
    if ((need_sorted || (flags & ECSIM_SORTED)) && !species[s].cell_start)
      return fail(ECSIM_EINVAL, "%s: cell_start is required for every species", who);
  }
  return ECSIM_OK;
}

}  // namespace

ecsim_status ecsim_moments(const ecsim_grid* grid, const ecsim_particles* species, int32_t nspecies,
                           const void* B_node, void* J, void* M, void* ws, size_t ws_bytes, uint32_t flags,
                           void* stream) {
  Grid g;
  SpeciesArgs a[kMaxSpecies];
  if (flags & ~(uint32_t)(ECSIM_ACCUMULATE | ECSIM_SORTED)) return fail(ECSIM_EINVAL, "ecsim_moments: unknown flags 0x%x", flags);
  if (species_list(grid, species, nspecies, g, a, "ecsim_moments", flags, false) != ECSIM_OK) return ECSIM_EINVAL;
  if (!B_node || !J || !M) return fail(ECSIM_EINVAL, "ecsim_moments: B_node, J and M are required");
  const bool f32 = species[0].prec == ECSIM_F32;
  const size_t esz = f32 ? 4 : 8;
  const bool tiled = (flags & ECSIM_SORTED) != 0;
  if (tiled && !tiled_species_ok(a, nspecies))
    return fail(ECSIM_EINVAL, "ecsim_moments: ECSIM_SORTED takes at most 4 species of fewer than 2^28 particles "
                              "each (without ECSIM_SORTED the any-order deposit takes more)");
  int64_t np_total = 0;
  for (int s = 0; s < nspecies; ++s) np_total += a[s].np;
  if (tiled) {
    const size_t need = tiled_workspace_bytes(g, np_total, f32);
    if (!ws || ws_bytes < need)
      return fail(ECSIM_EWORKSPACE, "ecsim_moments: workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : 0);
  }
  if (bind_flag(g, "ecsim_moments") != ECSIM_OK) return ECSIM_EHIP;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  const bool acc = (flags & ECSIM_ACCUMULATE) != 0;
  if (tiled) {
    // the tiled deposit's node flush writes (or adds to) every entry of J and M
    e = launch_deposit_tiled(g, f32, a, nspecies, B_node, J, M, acc, ws, st);
  } else {
    if (!acc) {
      if ((e = launch_zero(J, esz * 3 * (size_t)g.nn, st)) != hipSuccess) return hip_fail(e, "ecsim_moments zero J");
      if ((e = launch_zero(M, esz * 126 * (size_t)g.nn, st)) != hipSuccess) return hip_fail(e, "ecsim_moments zero M");
    }
    e = launch_deposit_atomic(g, f32, a, nspecies, B_node, J, M, st);
  }
  if (e != hipSuccess) return hip_fail(e, "ecsim_moments");
  return ECSIM_OK;
}

static size_t diag_ws_bytes(const Grid& g, bool f32, uint32_t flags) {
  if (flags & ECSIM_SORTED) return 256;            // a zero block
  return f32 ? sizeof(double) * 10 * (size_t)g.nn : 0;   // FP64 accumulators of the FP32 form
}

ecsim_status ecsim_diagnostics_workspace_size(const ecsim_grid* grid, int32_t prec, uint32_t flags, size_t* bytes) {
  Grid g;
  if (!bytes) return fail(ECSIM_EINVAL, "ecsim_diagnostics_workspace_size: bytes is NULL");
  if (make_grid(grid, g) != ECSIM_OK) return ECSIM_EINVAL;
  if (check_prec(prec) != ECSIM_OK) return ECSIM_EINVAL;
  if (flags & ~(uint32_t)(ECSIM_ACCUMULATE | ECSIM_SORTED))
    return fail(ECSIM_EINVAL, "ecsim_diagnostics_workspace_size: unknown flags 0x%x", flags);
  *bytes = diag_ws_bytes(g, prec == ECSIM_F32, flags);
  return ECSIM_OK;
}

ecsim_status ecsim_diagnostics(const ecsim_grid* grid, const ecsim_particles* species, int32_t nspecies, void* rho,
                               void* J, void* P, void* ws, size_t ws_bytes, uint32_t flags, void* stream) {
  Grid g;
  SpeciesArgs a[kMaxSpecies];
  if (flags & ~(uint32_t)(ECSIM_ACCUMULATE | ECSIM_SORTED))
    return fail(ECSIM_EINVAL, "ecsim_diagnostics: unknown flags 0x%x", flags);
  if (species_list(grid, species, nspecies, g, a, "ecsim_diagnostics", flags, false) != ECSIM_OK) return ECSIM_EINVAL;
  if (!rho || !J || !P) return fail(ECSIM_EINVAL, "ecsim_diagnostics: rho, J and P are required");
  const bool f32 = species[0].prec == ECSIM_F32;
  const size_t esz = f32 ? 4 : 8;
  const bool tiled = (flags & ECSIM_SORTED) != 0;
  if (tiled && !tiled_species_ok(a, nspecies))
    return fail(ECSIM_EINVAL, "ecsim_diagnostics: ECSIM_SORTED takes at most 4 species of fewer than 2^28 "
                              "particles each (without ECSIM_SORTED the any-order kernel takes more)");
  const size_t need = diag_ws_bytes(g, f32, tiled ? ECSIM_SORTED : 0);
  if (need && (!ws || ws_bytes < need))
    return fail(ECSIM_EWORKSPACE, "ecsim_diagnostics: workspace of %zu bytes needed, %zu given", need,
                ws ? ws_bytes : 0);
  if (bind_flag(g, "ecsim_diagnostics") != ECSIM_OK) return ECSIM_EHIP;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (!(flags & ECSIM_ACCUMULATE)) {
    if ((e = launch_zero(rho, esz * (size_t)g.nn, st)) != hipSuccess) return hip_fail(e, "ecsim_diagnostics zero rho");
    if ((e = launch_zero(J, esz * 3 * (size_t)g.nn, st)) != hipSuccess) return hip_fail(e, "ecsim_diagnostics zero J");
    if ((e = launch_zero(P, esz * 6 * (size_t)g.nn, st)) != hipSuccess) return hip_fail(e, "ecsim_diagnostics zero P");
  }
  if (tiled)
    e = launch_diagnostics_tiled(g, f32, a, nspecies, rho, J, P, ws, st);
  else
    e = launch_diagnostics_atomic(g, f32, a, nspecies, rho, J, P, ws, st);
  if (e != hipSuccess) return hip_fail(e, "ecsim_diagnostics");
  return ECSIM_OK;
}

ecsim_status ecsim_move_moments(const ecsim_grid* grid, const ecsim_particles* species, int32_t nspecies,
                                const void* E_node, const void* B_node, const void* B_next, void* J, void* M,
                                double* ke_out, void* ws, size_t ws_bytes, uint32_t flags, void* stream) {
  Grid g;
  SpeciesArgs a[kMaxSpecies];
  if (flags & ~(uint32_t)(ECSIM_ACCUMULATE | ECSIM_SORTED))
    return fail(ECSIM_EINVAL, "ecsim_move_moments: unknown flags 0x%x", flags);
  if (species_list(grid, species, nspecies, g, a, "ecsim_move_moments", flags, true) != ECSIM_OK) return ECSIM_EINVAL;
  if (!E_node || !B_node || !B_next || !J || !M)
    return fail(ECSIM_EINVAL, "ecsim_move_moments: E_node, B_node, B_next, J and M are required");
  if (!tiled_species_ok(a, nspecies))
    return fail(ECSIM_EINVAL, "ecsim_move_moments: at most 4 species of fewer than 2^28 particles each");
  int64_t np_total = 0;
  for (int s = 0; s < nspecies; ++s) np_total += a[s].np;
  const bool f32 = species[0].prec == ECSIM_F32;
  const size_t need = tiled_workspace_bytes(g, np_total, f32);
  if (!ws || ws_bytes < need)
    return fail(ECSIM_EWORKSPACE, "ecsim_move_moments: workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : 0);
  if (bind_flag(g, "ecsim_move_moments") != ECSIM_OK) return ECSIM_EHIP;
  hipStream_t st = (hipStream_t)stream;
  const hipError_t e = launch_move_deposit(g, f32, a, nspecies, E_node, B_node, B_next, J, M, ke_out,
                                           (flags & ECSIM_ACCUMULATE) != 0, ws, st);
  if (e != hipSuccess) return hip_fail(e, "ecsim_move_moments");
  return ECSIM_OK;
}

ecsim_status ecsim_move_moments_noalloc(const ecsim_grid* grid, const ecsim_particles* species, int32_t nspecies,
                                        const void* E_node, const void* B_node, const void* B_next, void* J,
                                        void* M, double* ke_out, uint32_t flags, void* stream) {
  const char* who = "ecsim_move_moments_noalloc";
  Grid g;
  SpeciesArgs a[kMaxSpecies];
  if (flags & ~(uint32_t)(ECSIM_ACCUMULATE | ECSIM_SORTED)) return fail(ECSIM_EINVAL, "%s: unknown flags 0x%x", who, flags);
  if (species_list(grid, species, nspecies, g, a, who, flags, true) != ECSIM_OK) return ECSIM_EINVAL;
  if (!E_node || !B_node || !B_next || !J || !M)
    return fail(ECSIM_EINVAL, "%s: E_node, B_node, B_next, J and M are required", who);
  if (!tiled_species_ok(a, nspecies))
    return fail(ECSIM_EINVAL, "%s: at most 4 species of fewer than 2^28 particles each", who);
  int64_t np_total = 0;
  for (int s = 0; s < nspecies; ++s) np_total += a[s].np;
  const bool f32 = species[0].prec == ECSIM_F32;
  const size_t need = tiled_workspace_bytes(g, np_total, f32);
  if (need > (size_t)ECSIM_NOALLOC_SCRATCH_BYTES)
    return fail(ECSIM_EWORKSPACE,
                "%s: %lld particles on %lld cells need %zu bytes of scratch; the static scratch holds %zu "
                "(use ecsim_move_moments with a workspace)",
                who, (long long)np_total, (long long)g.nn, need, (size_t)ECSIM_NOALLOC_SCRATCH_BYTES);
  void* ws = device_scratch();
  if (!ws) return fail(ECSIM_EHIP, "%s: the device's static scratch is not accessible", who);
  if (bind_flag(g, who) != ECSIM_OK) return ECSIM_EHIP;
  hipStream_t st = (hipStream_t)stream;
  // the same launches as ecsim_move_moments; every word of the scratch that
  // must start at zero (the stray counter, the zero block, the per-cell
  // counts) is cleared by those launches' own fill kernels, and the per-cell
  // sums are written before they are read
  const hipError_t e = launch_move_deposit(g, f32, a, nspecies, E_node, B_node, B_next, J, M, ke_out,
                                           (flags & ECSIM_ACCUMULATE) != 0, ws, st);
  if (e != hipSuccess) return hip_fail(e, who);
  return ECSIM_OK;
}

ecsim_status ecsim_move_moments_regroup(const ecsim_grid* grid, const ecsim_particles* species,
                                        const ecsim_particles* dst, int32_t nspecies, const void* E_node,
                                        const void* B_node, const void* B_next, void* J, void* M, double* ke_out,
                                        void* ws, size_t ws_bytes, uint32_t flags, void* stream) {
  const char* who = "ecsim_move_moments_regroup";
  Grid g;
  SpeciesArgs a[kMaxSpecies], d[kMaxSpecies];
  if (flags & ~(uint32_t)(ECSIM_ACCUMULATE | ECSIM_SORTED)) return fail(ECSIM_EINVAL, "%s: unknown flags 0x%x", who, flags);
  if (species_list(grid, species, nspecies, g, a, who, flags, true) != ECSIM_OK) return ECSIM_EINVAL;
  if (!dst) return fail(ECSIM_EINVAL, "%s: dst is NULL", who);
  if (!E_node || !B_node || !B_next || !J || !M)
    return fail(ECSIM_EINVAL, "%s: E_node, B_node, B_next, J and M are required", who);
  if (!tiled_species_ok(a, nspecies))
    return fail(ECSIM_EINVAL, "%s: at most 4 species of fewer than 2^28 particles each", who);
  if ((int64_t)nspecies * g.nn >= ((int64_t)1 << 31))
    return fail(ECSIM_EINVAL, "%s: species x cells = %lld exceeds 2^31 - 1", who, (long long)nspecies * g.nn);
  for (int s = 0; s < nspecies; ++s) {
    if (make_species(&dst[s], d[s], who) != ECSIM_OK) return ECSIM_EINVAL;
    if (dst[s].prec != species[s].prec || dst[s].np != species[s].np)
      return fail(ECSIM_EINVAL, "%s: dst[%d] differs from species[%d] in precision or size", who, s, s);
    if ((dst[s].q == nullptr) != (species[s].q == nullptr))
      return fail(ECSIM_EINVAL, "%s: dst[%d] and species[%d] differ in per-particle charge", who, s, s);
    if (!dst[s].cell_start) return fail(ECSIM_EINVAL, "%s: dst[%d].cell_start is required", who, s);
    // no target may alias a source array of any species
    const void* tg[9] = {dst[s].pos[0], dst[s].pos[1], dst[s].pos[2], dst[s].vel[0], dst[s].vel[1],
                         dst[s].vel[2], dst[s].q, dst[s].cell, dst[s].cell_start};
    for (int r = 0; r < nspecies; ++r) {
      const void* sr[9] = {species[r].pos[0], species[r].pos[1], species[r].pos[2], species[r].vel[0],
                           species[r].vel[1], species[r].vel[2], species[r].q, species[r].cell,
                           species[r].cell_start};
      for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j)
          if (tg[i] && tg[i] == sr[j]) return fail(ECSIM_EINVAL, "%s: dst[%d] aliases species[%d]", who, s, r);
    }
  }
  int64_t np_total = 0;
  for (int s = 0; s < nspecies; ++s) np_total += a[s].np;
  const bool f32 = species[0].prec == ECSIM_F32;
  const size_t need = tiled_workspace_bytes(g, np_total, f32);
  if (!ws || ws_bytes < need)
    return fail(ECSIM_EWORKSPACE, "%s: workspace of %zu bytes needed, %zu given", who, need, ws ? ws_bytes : 0);
  if (bind_flag(g, who) != ECSIM_OK) return ECSIM_EHIP;
  hipStream_t st = (hipStream_t)stream;
  const hipError_t e = launch_move_deposit_regroup(g, f32, a, d, nspecies, E_node, B_node, B_next, J, M, ke_out,
                                                   (flags & ECSIM_ACCUMULATE) != 0, ws, st);
  if (e != hipSuccess) return hip_fail(e, who);
  return ECSIM_OK;
}

ecsim_status ecsim_mass_apply(const ecsim_grid* grid, int32_t m_prec, const void* M, const double* x, double a,
                              double b, double* y, void* stream) {
  Grid g;
  if (make_grid(grid, g) != ECSIM_OK) return ECSIM_EINVAL;
  if (check_prec(m_prec) != ECSIM_OK) return ECSIM_EINVAL;
  if (!M || !x || !y) return fail(ECSIM_EINVAL, "ecsim_mass_apply: M, x and y are required");
  if ((const void*)x == (const void*)y) return fail(ECSIM_EINVAL, "ecsim_mass_apply: x and y must not alias");
  if (g.nn >= ((int64_t)1 << 29)) return fail(ECSIM_EINVAL, "ecsim_mass_apply: at most 2^29 - 1 cells");
  hipError_t e = launch_mass_apply(g, m_prec == ECSIM_F32, M, x, a, b, y, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ecsim_mass_apply");
  return ECSIM_OK;
}

ecsim_status ecsim_backward_workspace_size(const ecsim_grid* grid, int64_t np, int32_t prec, size_t* bytes) {
  Grid g;
  if (make_grid(grid, g) != ECSIM_OK) return ECSIM_EINVAL;
  if (np < 0) return fail(ECSIM_EINVAL, "ecsim_backward_workspace_size: np < 0");
  if (prec != ECSIM_F32 && prec != ECSIM_F64) return fail(ECSIM_EINVAL, "ecsim_backward_workspace_size: bad precision %d", prec);
  if (!bytes) return fail(ECSIM_EINVAL, "ecsim_backward_workspace_size: bytes is NULL");
  *bytes = backward_workspace_bytes(g, np, prec == ECSIM_F32);
  return ECSIM_OK;
}

ecsim_status ecsim_moments_backward(const ecsim_grid* grid, const ecsim_particles* sp, const void* E_node,
                                    const void* B_node, const void* gJ, const void* gM, void* gpos[3],
                                    void* gvel[3], void* gE, void* gB, void* ws, size_t ws_bytes, uint32_t flags,
                                    void* stream) {
  Grid g;
  SpeciesArgs a;
  if (make_grid(grid, g) != ECSIM_OK) return ECSIM_EINVAL;
  if (make_species(sp, a, "ecsim_moments_backward") != ECSIM_OK) return ECSIM_EINVAL;
  if (flags & ~(uint32_t)(ECSIM_BWD_THROUGH_MOVER | ECSIM_ACCUMULATE | ECSIM_BWD_OFFSET_GRAD))
    return fail(ECSIM_EINVAL, "ecsim_moments_backward: unknown flags 0x%x", flags);
  const bool through = flags & ECSIM_BWD_THROUGH_MOVER;
  const bool offset_grad = (flags & ECSIM_BWD_OFFSET_GRAD) != 0;
  if (offset_grad && sp->prec != ECSIM_F32)
    return fail(ECSIM_EINVAL, "ecsim_moments_backward: ECSIM_BWD_OFFSET_GRAD needs FP32 (offset + cell) particles");
  if (!B_node || !gJ || !gM || !gB) return fail(ECSIM_EINVAL, "ecsim_moments_backward: B_node, gJ, gM, gB are required");
  if (through && (!E_node || !gE)) return fail(ECSIM_EINVAL, "ecsim_moments_backward: through the mover needs E_node and gE");
  if (!gpos || !gvel) return fail(ECSIM_EINVAL, "ecsim_moments_backward: gpos and gvel are required");
  if (sp->np > 0)
    for (int d = 0; d < 3; ++d)
      if (!gpos[d] || !gvel[d]) return fail(ECSIM_EINVAL, "ecsim_moments_backward: gpos/gvel[%d] is NULL", d);
  if (a.cell_start && sp->np > 0) {
    const size_t need = backward_workspace_bytes(g, sp->np, sp->prec == ECSIM_F32);
    if (!ws || ws_bytes < need)
      return fail(ECSIM_EWORKSPACE, "ecsim_moments_backward: grouped particles need a workspace of %zu bytes, %zu given",
                  need, ws ? ws_bytes : (size_t)0);
  }
  if (bind_flag(g, "ecsim_moments_backward") != ECSIM_OK) return ECSIM_EHIP;
  hipError_t e = launch_backward(g, sp->prec == ECSIM_F32, a, E_node, B_node, gJ, gM, gpos, gvel, gE, gB, through,
                                 offset_grad, ws, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ecsim_moments_backward");
  return ECSIM_OK;
}

ecsim_status ecsim_sort(const ecsim_grid* grid, const ecsim_particles* src, const ecsim_particles* dst,
                        int32_t* cell_start_out, int32_t* perm_out, void* ws, size_t ws_bytes, void* stream) {
  Grid g;
  SpeciesArgs a, b;
  if (make_grid(grid, g) != ECSIM_OK) return ECSIM_EINVAL;
  if (make_species(src, a, "ecsim_sort src") != ECSIM_OK) return ECSIM_EINVAL;
  if (make_species(dst, b, "ecsim_sort dst") != ECSIM_OK) return ECSIM_EINVAL;
  if (src->prec != dst->prec || src->np != dst->np) return fail(ECSIM_EINVAL, "ecsim_sort: src and dst differ in precision or np");
  if ((src->q == nullptr) != (dst->q == nullptr)) return fail(ECSIM_EINVAL, "ecsim_sort: src and dst must both have or lack q");
  for (int d = 0; d < 3; ++d)
    if (src->np > 0 && (src->pos[d] == dst->pos[d] || src->vel[d] == dst->vel[d]))
      return fail(ECSIM_EINVAL, "ecsim_sort: src and dst arrays must not alias");
  if (!cell_start_out) return fail(ECSIM_EINVAL, "ecsim_sort: cell_start_out is required");
  size_t need = sort_workspace_bytes(g, src->np);
  if (!ws || ws_bytes < need) return fail(ECSIM_EWORKSPACE, "ecsim_sort: workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : 0);
  hipError_t e = launch_sort(g, src->prec == ECSIM_F32, a, b, cell_start_out, perm_out, ws, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ecsim_sort");
  return ECSIM_OK;
}

ecsim_status ecsim_centres_to_nodes(const ecsim_grid* grid, const double* B_C, double* B_N, float* B_N32,
                                    void* stream) {
  Grid g;
  if (make_grid(grid, g) != ECSIM_OK) return ECSIM_EINVAL;
  if (!B_C || (!B_N && !B_N32)) return fail(ECSIM_EINVAL, "ecsim_centres_to_nodes: B_C and an output are required");
  hipError_t e = launch_centres_to_nodes(g, B_C, B_N, B_N32, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ecsim_centres_to_nodes");
  return ECSIM_OK;
}

ecsim_status ecsim_to_f32(int64_t n, const double* src, float* dst, void* stream) {
  if (n < 0) return fail(ECSIM_EINVAL, "ecsim_to_f32: n < 0");
  if (n > 0 && (!src || !dst)) return fail(ECSIM_EINVAL, "ecsim_to_f32: NULL pointer");
  hipError_t e = launch_to_f32(n, src, dst, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ecsim_to_f32");
  return ECSIM_OK;
}

ecsim_status ecsim_field_energy(const ecsim_grid* grid, const double* F, double* out, void* ws, size_t ws_bytes,
                                void* stream) {
  Grid g;
  if (make_grid(grid, g) != ECSIM_OK) return ECSIM_EINVAL;
  if (!F || !out) return fail(ECSIM_EINVAL, "ecsim_field_energy: NULL pointer");
  if (!ws || ws_bytes < ECSIM_ENERGY_WS_BYTES)
    return fail(ECSIM_EWORKSPACE, "ecsim_field_energy: workspace of %d bytes needed", (int)ECSIM_ENERGY_WS_BYTES);
  hipError_t e = launch_sumsq(F, 3 * g.nn, g.V / (8.0 * kPi), (double*)ws, out, false, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ecsim_field_energy");
  return ECSIM_OK;
}

ecsim_status ecsim_check_finite(void* stream) {
  int* f = device_flag();
  if (!f) return fail(ECSIM_EHIP, "ecsim_check_finite: the device's non-finite flag is not accessible");
  hipError_t e;
  if ((e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess) return hip_fail(e, "ecsim_check_finite");
  int v = 0;
  if ((e = hipMemcpy(&v, f, sizeof v, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "ecsim_check_finite");
  if (v == 0) return ECSIM_OK;
  const int zero = 0;
  if ((e = hipMemcpy(f, &zero, sizeof zero, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "ecsim_check_finite");
  return fail(ECSIM_ENONFINITE, "a kernel produced a non-finite value since the last check");
}

ecsim_status ecsim_nonfinite_read(int32_t* flag_out, void* stream) {
  if (!flag_out) return fail(ECSIM_EINVAL, "ecsim_nonfinite_read: flag_out is NULL");
  int* f = device_flag();
  if (!f) return fail(ECSIM_EHIP, "ecsim_nonfinite_read: the device's non-finite flag is not accessible");
  hipError_t e = launch_take_flag(f, flag_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "ecsim_nonfinite_read");
  return ECSIM_OK;
}

// ---------------------------------------------------------------------------
// GMRES(m) field solve
// ---------------------------------------------------------------------------
ecsim_status ecsim_solve_workspace_size(const ecsim_grid* grid, int32_t restart, size_t* bytes) {
  Grid g;
  if (make_grid(grid, g) != ECSIM_OK) return ECSIM_EINVAL;
  if (restart < 1 || restart > kMaxRestart) return fail(ECSIM_EINVAL, "restart = %d not in 1..%d", restart, kMaxRestart);
  if (!bytes) return fail(ECSIM_EINVAL, "bytes is NULL");
  const size_t vec = align256(sizeof(double) * 3 * (size_t)g.nn);
  const size_t m = (size_t)restart, nb = (size_t)solve_blocks(g);
  // V (m + 1 vectors), two w buffers, the residual, b; the partial sums of
  // the two Gram-Schmidt passes and of |w|^2; the read-back block
  // (threshold, |r|, residual history, flags, partial |b|^2 and |r|^2); H,
  // the rotations, g, h1, h2 and the two least-squares solutions
  *bytes = vec * (m + 1) + 4 * vec + 2 * align256(sizeof(double) * nb * m) + align256(sizeof(double) * nb) +
           align256(sizeof(double) * (6 + m + 2 * nb)) + align256(sizeof(double) * ((m + 1) * m + 7 * m + 1));
  return ECSIM_OK;
}

namespace {
// steps the first batch of a solve launches before its first read-back:
// what the last solve's first cycle needed
std::atomic<int> g_first_batch{2};
}  // namespace

ecsim_status ecsim_field_solve(const ecsim_grid* grid, int32_t m_prec, const void* M, const void* J,
                               const double* E_n, const double* B_C_n, double tol, int32_t restart, int32_t maxit,
                               double* E_theta, double* E_next, double* B_C_next, void* ws, size_t ws_bytes,
                               int32_t* iters_out, double* resid_out, void* stream) {
  Grid g;
  if (make_grid(grid, g) != ECSIM_OK) return ECSIM_EINVAL;
  if (check_prec(m_prec) != ECSIM_OK) return ECSIM_EINVAL;
  if (!M || !J || !E_n || !B_C_n || !E_theta || !E_next || !B_C_next)
    return fail(ECSIM_EINVAL, "ecsim_field_solve: NULL array");
  if (!(tol > 0.0) || !(tol < 1.0)) return fail(ECSIM_EINVAL, "ecsim_field_solve: tol must be in (0, 1)");
  if (maxit < 1) return fail(ECSIM_EINVAL, "ecsim_field_solve: maxit must be >= 1");
  if (g.nn >= ((int64_t)1 << 29)) return fail(ECSIM_EINVAL, "ecsim_field_solve: at most 2^29 - 1 cells");
  size_t need = 0;
  if (ecsim_solve_workspace_size(grid, restart, &need) != ECSIM_OK) return ECSIM_EINVAL;
  if (!ws || ws_bytes < need) return fail(ECSIM_EWORKSPACE, "ecsim_field_solve: workspace of %zu bytes needed", need);

  const int m = restart;
  const int nb = solve_blocks(g);
  const size_t vec = align256(sizeof(double) * 3 * (size_t)g.nn);
  const int64_t ld = (int64_t)(vec / sizeof(double));
  char* w8 = (char*)ws;
  double* V = (double*)w8;
  w8 += vec * (size_t)(m + 1);
  double* Wb[2] = {(double*)w8, (double*)(w8 + vec)};
  w8 += 2 * vec;
  double* Wr = (double*)w8;
  w8 += vec;
  double* bvec = (double*)w8;
  w8 += vec;
  double* P1 = (double*)w8;
  w8 += align256(sizeof(double) * (size_t)nb * m);
  double* P2 = (double*)w8;
  w8 += align256(sizeof(double) * (size_t)nb * m);
  double* P3 = (double*)w8;
  w8 += align256(sizeof(double) * (size_t)nb);
  const size_t rb_count = 6 + (size_t)m + 2 * (size_t)nb;
  double* rb = (double*)w8;
  double* Pb = rb + 6 + m;
  double* Pr = Pb + nb;
  w8 += align256(sizeof(double) * rb_count);
  GmresState G;
  G.H = (double*)w8;
  G.cs = G.H + (size_t)(m + 1) * m;
  G.sn = G.cs + m;
  G.gv = G.sn + m;
  G.h1 = G.gv + (m + 1);
  G.h2 = G.h1 + m;
  G.yn = G.h2 + m;
  G.yp = G.yn + m;
  G.rb = rb;
  G.Pb = Pb;
  G.m = m;
  G.tol = tol;

  hipStream_t st = (hipStream_t)stream;
  const bool mf32 = m_prec == ECSIM_F32;
  const double ctd = kC * kTheta * g.dt, ctd2 = ctd * ctd, cm = 4.0 * kPi * kTheta * g.dt;
  CurlK K;
  curl_curl_stencil(g, ctd2, K);
  hipError_t e;
#define HIPCK(x)                                                 \
  do {                                                           \
    if ((e = (x)) != hipSuccess) return hip_fail(e, "ecsim_field_solve"); \
  } while (0)

  // Restarted GMRES(m), classical Gram-Schmidt applied twice, from E^n. A
  // step is three kernels (operator with the first pass's inner products,
  // first pass with the second's, second pass with the new norm); the
  // normalisation and the Givens update of H and g ride on the next step's
  // first kernel, and every inner product is summed by the kernel that needs
  // it. Steps go out in batches, and every batch ends as if it closed the
  // solve: y over the columns so far, X moved by V times the change in y,
  // the true residual and the field advance. The host reads back once per
  // batch; if the residual is not yet below tol it launches more steps of
  // the same cycle (or, once the cycle has m columns or its estimate has
  // converged, a new cycle from the residual just computed). The first
  // batch is as long as the last solve's first cycle, later ones as long as
  // the observed convergence rate predicts; steps past convergence change
  // nothing.
  std::vector<double> hb(rb_count);
  auto read_back = [&]() -> hipError_t {
    hipError_t r = hipMemcpyAsync(hb.data(), rb, sizeof(double) * rb_count, hipMemcpyDeviceToHost, st);
    return r != hipSuccess ? r : hipStreamSynchronize(st);
  };
  auto host_sum = [&](size_t off) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += hb[off + b];
    return s;
  };
  const size_t off_pb = 6 + (size_t)m, off_pr = off_pb + nb;
  const int* flags = (const int*)(hb.data() + 4 + m);
  const double* hh = hb.data() + 4;

  HIPCK(launch_residual_first(g, mf32, M, K, cm, E_n, J, B_C_n, -4.0 * kPi * kTheta * g.dt, ctd, bvec, E_theta, Wr,
                              Pb, Pr, st));
  int it_done = 0;    // columns of the cycles before this one
  int it = 0;
  int j = 0;          // steps launched in this cycle
  double rel = 0.0, bnorm = 0.0;
  bool converged = false, first = true;
  int batch = std::max(1, std::min(g_first_batch.load(std::memory_order_relaxed), m));
  while (true) {
    const int nbat = std::min(std::min(batch, m - j), maxit - it_done - j);
    for (int s = j; s < j + nbat; ++s) {
      const int mode = s == 0 ? kArnoldiStart : (s > j ? kArnoldiGivens : kArnoldiNone);
      double* w = Wb[(s + 1) & 1];
      HIPCK(launch_arnoldi_op(g, mf32, M, K, cm, s == 0 ? Wr : Wb[s & 1], w, V, ld, s, mode, s == 0 ? Pr : P3,
                              P1, G, st));
      HIPCK(launch_cgs_pass(g, false, V, ld, s + 1, P1, G.h1, w, P2, st));
      HIPCK(launch_cgs_pass(g, true, V, ld, s + 1, P2, G.h2, w, P3, st));
    }
    HIPCK(launch_givens_tail(g, j + nbat - 1, P3, G, st));
    HIPCK(launch_update_x(g, V, ld, E_theta, G, st));
    HIPCK(launch_residual_last(g, mf32, M, K, cm, E_theta, bvec, Wr, Pr, E_n, B_C_n, ctd, E_next, B_C_next, G, st));
    HIPCK(read_back());
    if (first) {
      const double bb = host_sum(off_pb);
      if (!std::isfinite(bb))
        return fail(ECSIM_ENONFINITE, "ecsim_field_solve: the right-hand side is not finite (J, E^n or B^n)");
      bnorm = std::sqrt(bb);
      first = false;
      if (bnorm == 0.0) {
        // b = 0: E^{n+theta} = 0
        HIPCK(launch_zero(E_theta, sizeof(double) * 3 * (size_t)g.nn, st));
        HIPCK(launch_finish(g, E_n, E_theta, B_C_n, ctd, E_next, B_C_next, nullptr, st));
        HIPCK(hipStreamSynchronize(st));
        converged = true;
        break;
      }
    }
    if (j == 0 && !std::isfinite(hb[1]))
      return fail(ECSIM_ENONFINITE, "ecsim_field_solve: the residual is not finite (M or the iterate)");
    for (int s = j; s < j + nbat; ++s)
      if (!std::isfinite(hh[s]))
        return fail(ECSIM_ENONFINITE, "ecsim_field_solve: a Krylov vector is not finite (M is not finite)");
    j += nbat;
    const int used = flags[1];
    it = it_done + used;
    rel = std::sqrt(host_sum(off_pr)) / bnorm;
    if (!std::isfinite(rel))
      return fail(ECSIM_ENONFINITE, "ecsim_field_solve: the residual is not finite (M or the iterate)");
    if (it_done == 0 && used > 0) g_first_batch.store(used, std::memory_order_relaxed);
    if (rel <= tol) {
      converged = true;
      break;
    }
    if (it_done + j >= maxit) break;
    if (flags[0] == 0 || j >= m) {
      // a new cycle from the residual of the iterate
      if (used == 0) break;   // no progress possible
      it_done += used;
      j = 0;
      batch = std::max(1, std::min(g_first_batch.load(std::memory_order_relaxed), m));
      continue;
    }
    // steps still needed at the rate of the last two: |g| falls by about
    // hist[j-1] / hist[j-2] per step
    int next = 1;
    if (j >= 2 && hh[j - 1] > 0.0 && hh[j - 2] > hh[j - 1]) {
      const double rate = hh[j - 1] / hh[j - 2];
      const double k = std::log(hb[0] / hh[j - 1]) / std::log(rate);
      next = k < 1.0 ? 1 : (k > (double)m ? m : (int)std::ceil(k));
    }
    batch = next;
  }
#undef HIPCK
  if (iters_out) *iters_out = it;
  if (resid_out) *resid_out = rel;
  if (!converged) return fail(ECSIM_ENOCONV, "ecsim_field_solve: relative residual %.3e after %d iterations", rel, it);
  return ECSIM_OK;
}

}  // extern "C"
