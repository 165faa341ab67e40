/*
 * ecsim.h -- C ABI of the MI355X (gfx950) ECsim particle hot path.
 *
 * The semi-implicit, energy-conserving PIC scheme (ECsim) advances, per time
 * step: moment gathering (hatted current J-hat, Eq. 1; mass matrices M, Eq. 3),
 * the implicit field solve (Eqs. 6-7, GMRES) and the particle mover
 * (Eqs. 4, 5, 8). This library implements those steps as HIP kernels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Units: Gaussian with the 4 pi factor, c = 1, theta = 1/2 (the value the
 *    paper states gives energy conservation, Sec. II).
 *  - Grid: periodic, n[d] cells of size h[d]; nodes sit at i*h, cell i spans
 *    [i h, (i+1) h). Node and cell index: ix + nx*(iy + ny*iz). Every node has
 *    the control volume V = hx*hy*hz.
 *  - Node fields (E, B at nodes, J-hat, gradients) are [3][Nn] structure of
 *    arrays. Cell-centred B_C is [3][Nc] with the index of the cell.
 *  - Mass matrices are stored as 14 offset blocks per node, [14][9][Nn]:
 *    block k of node g is M_{g, g+o_k}; component ij = 3*i + j. The 14 offsets
 *    o_k are (0,0,0); (1,0,0); (ox,1,0) for ox = -1,0,1; and (ox,oy,1) with ox
 *    fastest and oy, ox in -1..1 (Eq. 3 and the symmetry M_{NN'} = M_{N'N}
 *    stated after it: the 13 offsets not stored satisfy M_{g,g-o} = M_{g-o,g},
 *    which is block k of node g-o).
 *  - Every pointer to an array is a DEVICE pointer owned by the caller, except
 *    where marked "host". The library never frees caller memory. Calls are
 *    asynchronous on `stream` (a hipStream_t; NULL is the default stream)
 *    unless marked "synchronous".
 *  - Arguments are validated on the host before anything is launched; a bad
 *    argument returns ECSIM_EINVAL and launches nothing. A HIP launch or
 *    runtime failure returns ECSIM_EHIP. ecsim_last_error() describes the last
 *    non-OK status of the calling thread. Nothing throws across this ABI.
 *  - Non-finite values: the kernels of the mover, the moment deposits, the
 *    diagnostics and the adjoint set a per-device flag when they produce a
 *    NaN or an infinity (new velocities, deposited node values, gradients);
 *    no call synchronises to look at it. ecsim_check_finite() (synchronous)
 *    and ecsim_nonfinite_read() (asynchronous) report and clear it.
 *  - Precision: ECSIM_F64 particles use FP64 fields and outputs. ECSIM_F32
 *    particles store an int32 cell index plus FP32 in-cell offsets in [0,1)
 *    and FP32 velocities and use FP32 node fields. Their arithmetic: the
 *    mover gathers E and B and pushes positions in FP32 but forms the
 *    rotation alpha_p and the velocity update v^{n+1} = 2 alpha_p u - v^n in
 *    FP64, rounding v^{n+1} once to FP32 (an FP32 alpha_p would scale |v| by
 *    the same 1 + O(1e-7) for every particle in a uniform B, a one-way energy
 *    drift). The moment deposits form alpha_p, the weights and J-hat and M in
 *    FP32. The grouped (ECSIM_SORTED) deposit sums a cell's particles in
 *    blocks of 64 on the matrix cores (plain FP32 sums inside a block) and
 *    combines the blocks with Kahan compensation, then adds each node value
 *    to J and M with one FP32 atomic per brick of cells; the any-order
 *    deposit adds every particle's terms with plain FP32 atomics.
 */
#ifndef ECSIM_H
#define ECSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ecsim_status;
enum {
  ECSIM_OK = 0,
  ECSIM_EINVAL = -1,       /* invalid argument (nothing launched)            */
  ECSIM_EHIP = -2,         /* HIP runtime or launch error                    */
  ECSIM_EWORKSPACE = -3,   /* workspace missing or smaller than required     */
  ECSIM_ENONFINITE = -4,   /* a NaN or infinity was produced (see above)     */
  ECSIM_ENOCONV = -5       /* GMRES did not reach the tolerance              */
};

enum { ECSIM_F64 = 0, ECSIM_F32 = 1 };

/* flags */
enum {
  ECSIM_ACCUMULATE = 1,    /* add into J/M (or gE/gB) instead of overwriting */
  ECSIM_SORTED = 2,        /* particles are grouped by cell; cell_start valid */
  ECSIM_BWD_THROUGH_MOVER = 8, /* backward: differentiate mover -> moments  */
  ECSIM_BWD_OFFSET_GRAD = 16   /* backward, FP32 only: gpos = dL/d(offset)    */
};

typedef struct {
  int32_t n[3];            /* cells per dimension, >= 1                      */
  double h[3];             /* cell size, > 0                                  */
  double dt;               /* time step, > 0                                  */
} ecsim_grid;

/* One species. All arrays have np entries and live on the device. */
typedef struct {
  int32_t prec;            /* ECSIM_F64 or ECSIM_F32                          */
  int64_t np;              /* number of particles, 0 <= np < 2^31             */
  double qom;              /* charge-to-mass ratio (q/m) of the species        */
  void *pos[3];            /* F64: absolute position in [0, n*h);
                              F32: in-cell offset in [0, 1)                   */
  int32_t *cell;           /* F32: cell index of the particle; F64: NULL       */
  void *vel[3];            /* velocity components (prec)                      */
  const void *q;           /* per-particle charge (prec), or NULL             */
  double q_const;          /* charge of every particle when q == NULL         */
  const int32_t *cell_start; /* optional, with ECSIM_SORTED: [Nc+1] offsets of
                              each cell's particles (particles of cell c are
                              [cell_start[c], cell_start[c+1]))               */
} ecsim_particles;

/* Thread-local description of the last non-OK status (never NULL). */
const char *ecsim_last_error(void);

/* Library version string (host). */
const char *ecsim_version(void);

/*
 * Non-finite values (a NaN or an infinity in an input propagates to the new
 * velocities, the deposited J-hat, M and diagnostic values, or the adjoint's
 * particle gradients, where the kernels record it in a per-device flag):
 *   ecsim_check_finite: synchronous. Waits for `stream`, reads the current
 *     device's flag and clears it; returns ECSIM_ENONFINITE if any kernel of
 *     this library on the device (any stream) produced a non-finite value
 *     since the flag was last cleared, else ECSIM_OK.
 *   ecsim_nonfinite_read: asynchronous on `stream`; copies the flag into the
 *     device int32 *flag_out (0 = all finite, 1 = a non-finite value seen) and
 *     clears it, in stream order.
 * The field solve reports a non-finite right-hand side or residual itself
 * (ECSIM_ENONFINITE). The flag is per device and shared by every stream.
 */
ecsim_status ecsim_check_finite(void *stream);
ecsim_status ecsim_nonfinite_read(int32_t *flag_out /* device */, void *stream);

/* Bytes of device workspace that ecsim_sort, ecsim_moments (with
 * ECSIM_SORTED), ecsim_move_moments and ecsim_move_moments_regroup need for
 * `np` particles in total (all species of one call) of precision `prec` on
 * this grid (host, synchronous). */
ecsim_status ecsim_workspace_size(const ecsim_grid *grid, int64_t np, int32_t prec,
                                  uint32_t flags, size_t *bytes /* host out */);

/*
 * The charge-to-mass ratio with which the kernels of precision `prec` move a
 * species of ratio `qom` (host, synchronous): they carry beta = qom dt / 2 as
 * a constant of that precision (the beta_p of Eqs. 2 and 4-5), so
 * *out = 2 beta / dt, which in ECSIM_F32 differs from qom by the FP32
 * rounding of beta (1.5e-8 relative for qom = -1, dt = 0.1). The scheme
 * conserves the total energy of the particles it moves (Secs. I-II, theta =
 * 1/2): every kinetic energy this library returns (ke_out) uses the masses
 * m_p = q_p / *out, and a caller that sums the kinetic energy itself should
 * too; with q_p / qom the FP32 total drifts one way by that rounding times the
 * work the field does on the species.
 */
ecsim_status ecsim_species_qom(int32_t prec, double qom, double dt, double *out /* host */);

/*
 * Particle mover, Eqs. 4, 5 and 8 of the paper:
 *   E_p, B_p = trilinear gathers of E_node = E^{n+theta} and B_node = B^n at
 *              x^{n-1/2};
 *   vbar     = alpha_p (v^n + beta_p E_p), alpha_p from Eq. 2 with beta_p =
 *              (q/m) dt / 2;
 *   v^{n+1}  = 2 vbar - v^n;  x^{n+1/2} = x^{n-1/2} + dt v^{n+1}, wrapped into
 *              the periodic box (F32: offset and cell updated).
 * Along a dimension of a single cell (a reduced 1D or 2D run) positions are
 * not pushed: the mover's fixPosition step (Sec. III) keeps particles on
 * their line or plane; velocities keep all three components. The same holds
 * in ecsim_move_moments and in the adjoint through the mover.
 * Updates pos/cell/vel of `sp` in place, preserving particle order.
 * E_node, B_node: [3][Nn] in the particles' precision.
 * ke_out: optional device double; receives (+=) sum_p 1/2 m_p |v^{n+1}|^2 with
 * m_p = q_p / (q/m)_int, (q/m)_int from ecsim_species_qom for the particles'
 * precision. Per-particle charges are read only for ke_out.
 */
ecsim_status ecsim_move(const ecsim_grid *grid, const ecsim_particles *sp,
                        const void *E_node, const void *B_node, double *ke_out,
                        void *stream);

/*
 * Moment gather, Eqs. 1 and 3 of the paper, summed over `nspecies` species:
 *   J[g]    = sum_p q_p (alpha_p v_p) W_pg / V                      [3][Nn]
 *   M[g][k] = sum_p (beta_p q_p / V) alpha_p W_pg W_p(g+o_k)    [14][9][Nn]
 * with alpha_p built from B_node (= B^n, [3][Nn]) gathered at x_p.
 * All species must share one precision; J, M and B_node are in it.
 * J and M are overwritten unless ECSIM_ACCUMULATE is set. With ECSIM_SORTED
 * every species must carry cell_start (particles grouped by cell ranges) and
 * the tiled deposit is used (at most 4 species of fewer than 2^28 particles
 * each, else ECSIM_EINVAL); a particle that is not in its range's cell is
 * still deposited correctly, through a slower stray path. Without
 * ECSIM_SORTED a per-particle atomic deposit handles any order and any
 * number of species.
 * ws/ws_bytes: with ECSIM_SORTED, device workspace of at least
 * ecsim_workspace_size() bytes for the total particle count; else unused.
 */
ecsim_status ecsim_moments(const ecsim_grid *grid, const ecsim_particles *species,
                           int32_t nspecies, const void *B_node, void *J, void *M,
                           void *ws, size_t ws_bytes, uint32_t flags, void *stream);

/*
 * Diagnostic moments of the output routines (paper, Sec. III: the diagnostics
 * computed for I/O, charge density, charge current and pressure tensor),
 * summed over `nspecies` species at the particles' stored positions and
 * velocities, with the interpolation weights W_pg of the moment gather:
 *   rho[g]  = sum_p q_p W_pg / V                                       [Nn]
 *   J[c][g] = sum_p q_p v_c W_pg / V  (no velocity rotation)        [3][Nn]
 *   P[k][g] = sum_p q_p v_i v_j W_pg / V, (i, j) = xx, xy, xz, yy, yz, zz
 *             for k = 0..5 (charge-weighted second velocity moment)  [6][Nn]
 * All species share one precision; rho, J and P are in it and are
 * overwritten unless ECSIM_ACCUMULATE is set. With ECSIM_SORTED every species
 * carries cell_start and a tiled kernel is used (a particle outside its
 * range's cell is still counted, through a slower path; at most 4 species of
 * fewer than 2^28 particles each, else ECSIM_EINVAL). Without
 * ECSIM_SORTED a per-particle atomic kernel takes any order; its FP32 form
 * accumulates in FP64 in the workspace and rounds once into the outputs.
 * ws/ws_bytes: device workspace of ecsim_diagnostics_workspace_size() bytes
 * for the same precision and flags (may be 0 and NULL); contents not kept.
 * Errors: ECSIM_EINVAL for bad arguments or flags, ECSIM_EWORKSPACE for a
 * missing or short workspace.
 */
ecsim_status ecsim_diagnostics_workspace_size(const ecsim_grid *grid, int32_t prec, uint32_t flags,
                                              size_t *bytes);
ecsim_status ecsim_diagnostics(const ecsim_grid *grid, const ecsim_particles *species,
                               int32_t nspecies, void *rho, void *J, void *P,
                               void *ws, size_t ws_bytes, uint32_t flags, void *stream);

/*
 * Fused particle pass of one step: every species is moved as by ecsim_move
 * (E_node = E^{n+theta}, B_node = B^n, Eqs. 4, 5, 8), then the moments of
 * Eqs. 1 and 3 at the new positions with B_next = B^{n+1} (the next step's
 * moment gather) are deposited into J and M, summed over species, as by
 * ecsim_moments with ECSIM_SORTED. Every species must carry cell_start; the
 * grouping may be stale (particles out of their range's cell take a slower
 * path), so a re-sort every few steps keeps the pass fast. Particles keep
 * their array positions. ke_out (nullable, device double) += the kinetic
 * energy of v^{n+1}. At most 4 species of fewer than 2^28 particles each.
 * ws: device workspace of ecsim_workspace_size() bytes for the total count.
 */
ecsim_status ecsim_move_moments(const ecsim_grid *grid, const ecsim_particles *species,
                                int32_t nspecies, const void *E_node, const void *B_node,
                                const void *B_next, void *J, void *M, double *ke_out,
                                void *ws, size_t ws_bytes, uint32_t flags, void *stream);

/*
 * ecsim_move_moments without a workspace argument and without any device
 * allocation, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc. The
 * scratch (stray list, stray state, per-cell counts and their scan) is a
 * static device array of ECSIM_NOALLOC_SCRATCH_BYTES that the library holds
 * on every device it runs on until the process ends; every call clears what
 * must start at zero. Calls on one device share that array, so two calls
 * that overlap on one GPU (different streams, or threads) race and give
 * wrong results; serialise them. Moves, J, M, ke_out, flags and errors as
 * for ecsim_move_moments; ECSIM_EWORKSPACE (nothing launched) when the
 * particles and grid need more scratch than the array holds: the bytes
 * ecsim_workspace_size reports for the total particle count must not exceed
 * ECSIM_NOALLOC_SCRATCH_BYTES (about 800,000 FP32 or 480,000 FP64 particles
 * on small grids). Allocates nothing, calls no allocating routine.
 */
#define ECSIM_NOALLOC_SCRATCH_BYTES (64u << 20)
ecsim_status ecsim_move_moments_noalloc(const ecsim_grid *grid, const ecsim_particles *species,
                                        int32_t nspecies, const void *E_node, const void *B_node,
                                        const void *B_next, void *J, void *M, double *ke_out,
                                        uint32_t flags, void *stream);

/*
 * The fused particle pass of ecsim_move_moments (same moves, same J and M),
 * which also regroups the particles by cell for the next pass: the deposit
 * takes every particle cell by cell (a cell's own range particles still in
 * it, then the particles that arrived), and writes each species' particles in
 * that order to dst[s], whose cell_start receives the new ranges. The paper
 * does not sort its particles (Sec. III); here the grouping that the tiled
 * deposit relies on is renewed at the cost of one more write of the particle
 * state, in place of a separate sort. Called every few steps (ecsim_move_moments
 * in between, on the grouping as it goes stale) it costs least per step.
 *   species: as for ecsim_move_moments (grouped, cell_start required); their
 *            arrays are moved in place and are no longer grouped afterwards.
 *   dst:     nspecies targets (device arrays) of the same precision and sizes,
 *            with a per-particle charge array exactly where the source has
 *            one, a cell array in the FP32 form and a cell_start of
 *            cells + 1 int32 (device out); none may alias a source array.
 *            After the call dst[s] holds species s's moved particles in cell
 *            order (positions, velocities, charges, cells) and is what the
 *            next pass takes as `species`.
 * Needs nspecies * cells < 2^31. Workspace, flags, ke_out and errors as for
 * ecsim_move_moments (ECSIM_EINVAL also for a mismatched or aliasing target).
 */
ecsim_status ecsim_move_moments_regroup(const ecsim_grid *grid, const ecsim_particles *species,
                                        const ecsim_particles *dst, int32_t nspecies,
                                        const void *E_node, const void *B_node, const void *B_next,
                                        void *J, void *M, double *ke_out, void *ws, size_t ws_bytes,
                                        uint32_t flags, void *stream);

/*
 * Matrix-free mass-matrix apply inside the field solve (Eq. 7):
 *   y = a * (M x) + b * y,   (M x)_g = sum over the 27 neighbours g' of
 *   M_{g g'} x_{g'}, using the 14 stored blocks and M_{g,g-o} = M_{g-o,g}
 *   (identical, not transposed, blocks).
 * M: [14][9][Nn] in precision m_prec; x, y: FP64 [3][Nn]; x and y must not
 * alias. Arithmetic is FP64. Grids of fewer than 2^29 cells, else ECSIM_EINVAL.
 */
ecsim_status ecsim_mass_apply(const ecsim_grid *grid, int32_t m_prec, const void *M,
                              const double *x, double a, double b, double *y,
                              void *stream);

/*
 * Adjoint of (mover ->) moments for the scalar L = <gJ, J> + <gM, M>, where J
 * and M are the moments of Eqs. 1 and 3 over the 14 stored blocks.
 * `sp` holds the particle state the forward started from. With
 * ECSIM_BWD_THROUGH_MOVER the forward is x', v' = mover(x, v; E_node, B_node)
 * followed by moments(x', v'; B_node) (same B_node); without it the forward is
 * moments(x, v; B_node) and E_node may be NULL.
 * Outputs: gpos[3], gvel[3] per particle, dL/d(position) and dL/d(velocity),
 * in the particles' precision. The position derivative is with respect to the
 * physical coordinate; with ECSIM_BWD_OFFSET_GRAD (FP32 particles only, else
 * ECSIM_EINVAL) it is with respect to the stored in-cell offset instead, i.e.
 * h times the physical one. gE, gB: [3][Nn], accumulated
 * (+=) always; gE untouched without ECSIM_BWD_THROUGH_MOVER. gJ: [3][Nn],
 * gM: [14][9][Nn], in the particles' precision. Alpha and the weights are
 * recomputed, not stored.
 * If sp->cell_start is set (particles grouped by cell ranges), a brick-tiled
 * kernel forms each cell's table of gradient blocks once (the 36 stored corner
 * pairs of gM summed by weight class, and gJ at the 8 corners) and handles the
 * particles that stay in their range's cell; the others (stale grouping, or
 * leaving the cell in the move) are listed in ws and handled one thread each,
 * with their post-move cell's table read from ws. ws is then required: device
 * workspace of ecsim_backward_workspace_size() bytes (else ECSIM_EWORKSPACE);
 * without cell_start ws is unused (may be NULL). Calls that share a workspace
 * must not overlap.
 */
ecsim_status ecsim_moments_backward(const ecsim_grid *grid, const ecsim_particles *sp,
                                    const void *E_node, const void *B_node,
                                    const void *gJ, const void *gM, void *gpos[3],
                                    void *gvel[3], void *gE, void *gB,
                                    void *ws, size_t ws_bytes, uint32_t flags, void *stream);

/*
 * Workspace of ecsim_moments_backward for np particles of precision prec
 * grouped by cell: the list count, a list of np indices and a table of 268
 * values per cell, in bytes. ECSIM_EINVAL for a bad grid, np < 0, an unknown
 * precision or a NULL bytes.
 */
ecsim_status ecsim_backward_workspace_size(const ecsim_grid *grid, int64_t np, int32_t prec, size_t *bytes);

/*
 * Counting sort of one species by cell, out of place. The paper's moment
 * gather runs over particles in storage order with atomic updates; its
 * authors tried sorting the particles (with reductions) and dropped it
 * (Sec. III). Here grouping by cell is what lets the tiled deposit reduce a
 * cell's particles before touching memory, and this call is the explicit
 * sort. The particles of `src` are written to the arrays of `dst` (same
 * precision and np, no aliasing) in cell order; the order inside a cell is
 * not specified. cell_start_out [Nc+1] receives each cell's range in dst and,
 * if perm_out is not NULL, perm_out[i] (int32) the index in src of the
 * particle now at dst[i]. ws: device workspace of ecsim_workspace_size() bytes.
 */
ecsim_status ecsim_sort(const ecsim_grid *grid, const ecsim_particles *src,
                        const ecsim_particles *dst, int32_t *cell_start_out,
                        int32_t *perm_out, void *ws, size_t ws_bytes, void *stream);

/* Node magnetic field: B_N[g] = mean of the 8 cell-centred values around node
 * g (FP64 in, FP64 out; B_N32 optional FP32 copy). */
ecsim_status ecsim_centres_to_nodes(const ecsim_grid *grid, const double *B_C, double *B_N,
                                    float *B_N32, void *stream);

/* FP64 -> FP32 copy of n values (node fields for the FP32 path). */
ecsim_status ecsim_to_f32(int64_t n, const double *src, float *dst, void *stream);

/*
 * Field solve of Eqs. 6-7 for theta = 1/2 (synchronous on `stream`):
 *   A E = b,  A E = E + (c theta dt)^2 curl_N curl_C E + 4 pi theta dt (M E),
 *   b = E^n - 4 pi theta dt J + c theta dt curl_N B_C^n,
 * by restarted GMRES(restart), 1 <= restart <= 120, from E^n, stopping when ||b - A E||_2 <=
 * tol ||b||_2 (grids of fewer than 2^29 cells, else ECSIM_EINVAL); then B_C^{n+theta} = B_C^n - c theta dt curl_C E^{n+theta},
 * E^{n+1} = 2 E^{n+theta} - E^n and B_C^{n+1} = 2 B_C^{n+theta} - B_C^n.
 * The curls average the four edge differences of a cell (curl_C, nodes to
 * centres) or the four around a node (curl_N, centres to nodes); curl_N is the
 * transpose of curl_C. M [14][9][Nn] and J [3][Nn] in m_prec (the precision
 * of the moments); every other vector FP64 [3][Nn]; the arithmetic is FP64.
 * ws: device workspace of ecsim_solve_workspace_size() bytes.
 * iters_out, resid_out (host, nullable): iterations and final relative
 * residual. Returns ECSIM_ENOCONV if maxit iterations did not reach tol (the
 * outputs then hold the last iterate). The Arnoldi steps run on the device in
 * batches; the host reads back once per batch (once per call when the call
 * needs as many steps as the previous call in the process needed at its
 * start), and the returned residual is the true one, ||b - A E|| / ||b||.
 */
ecsim_status ecsim_solve_workspace_size(const ecsim_grid *grid, int32_t restart, size_t *bytes);
ecsim_status ecsim_field_solve(const ecsim_grid *grid, int32_t m_prec, const void *M,
                               const void *J, const double *E_n, const double *B_C_n,
                               double tol, int32_t restart, int32_t maxit, double *E_theta,
                               double *E_next, double *B_C_next, void *ws, size_t ws_bytes,
                               int32_t *iters_out, double *resid_out, void *stream);

/* out (device double) = V/(8 pi) * sum over the 3*Nn values of F^2: the
 * field energy of an FP64 [3][Nn] array, the W_E and W_B terms of the total
 * energy the scheme conserves for theta = 1/2 (Sec. I-II). Deterministic
 * (fixed-order tree reduction). ws: device scratch of ECSIM_ENERGY_WS_BYTES. */
#define ECSIM_ENERGY_WS_BYTES 2048
ecsim_status ecsim_field_energy(const ecsim_grid *grid, const double *F, double *out,
                                void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ECSIM_H */
