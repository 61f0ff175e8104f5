/*
 * obem.h -- C ABI of the MI355X (gfx950) space-charge field library.
 *
 * The library implements the per-tracking-step field re-evaluation of
 * OuroborosBEM (arXiv 2110.09214): the field of the BEM surface-charge cells
 * (eqs. (BEM2), (BEM3)) plus the direct pairwise Coulomb field of the charged
 * particles (eq. (nbody)), the FP64 collocation solve that gives the cell
 * charges (eq. (matrixBEM)), the Euler push with null-collision Monte Carlo
 * that consumes the field (sections 3.3.5, 3.4), and an adjoint of the field
 * evaluation.
 *
 * General conventions
 *  - Units are SI: m, V, C, kg, s; cell charge densities sigma in C/m^2.
 *  - Every array argument is a DEVICE pointer (allocated by the caller on the
 *    context's device, e.g. a torch tensor's data_ptr()) unless it is marked
 *    "host".  The caller owns every array it passes; the library never frees
 *    or keeps a caller pointer after a call returns.  Arrays are contiguous,
 *    structure-of-arrays (one array per coordinate), float64 unless stated.
 *  - Calls are asynchronous on the context's HIP stream, except where a host
 *    output (info / stats) is requested, which synchronises the stream.
 *  - Arguments are validated on the host before any launch (NULL pointers,
 *    negative or too large sizes, pointers that are not device memory, soft <
 *    0, ...): OBEM_EINVAL, with a message in obem_last_error().  A failed HIP
 *    call returns OBEM_EDEVICE and leaves the context unusable (sticky); it
 *    must then be destroyed.
 *  - A context is not thread-safe: one host thread at a time per context.
 *    Sizes are int64_t but each particle/target/source/cell count must be
 *    below 2^31.
 */
#ifndef OBEM_H
#define OBEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OBEM_OK = 0,
  OBEM_EINVAL = -1,     /* invalid argument (nothing launched)                 */
  OBEM_ENOMEM = -2,     /* device allocation failed                            */
  OBEM_EDEVICE = -3,    /* HIP runtime / library error (sticky)                */
  OBEM_ESINGULAR = -4,  /* zero pivot in the LU factorisation                  */
  OBEM_ENOCONV = -5,    /* refinement did not reach the backward-error target  */
  OBEM_ECAPACITY = -6,  /* particle buffer too small; children dropped         */
  OBEM_ESTATE = -7      /* call made on a context in the sticky error state    */
} obem_status;

typedef enum {
  OBEM_FP64 = 0,   /* every sum and integral in float64: cells nearer than 48
                      diameters by the closed-form integrals, farther ones by
                      a 7-point rule; pairwise terms and sums in float64      */
  OBEM_MIXED = 1   /* cells nearer than 3 diameters: float64 closed-form
                      integrals.  Farther cells: float32 quadrature of the
                      cell (7 points within 6 diameters, 6 within 16, 4
                      within 40, 3 beyond, each rule's truncation error
                      below the float32 rounding floor; a group of 64
                      targets takes the finest rule one of them may need;
                      the same in the influence and the adjoint).
                      Pairwise terms in
                      float32 from coordinates
                      recentred near the targets (float32 hi + lo pairs for
                      the sources near them, so close pairs keep their
                      separation exactly).  Sums: float32 over blocks of
                      sources (one 256-source tile, or with targets = sources
                      the 2048-particle super-blocks of the pair-once
                      evaluation), the blocks added with compensation or in
                      float64 in a fixed order; nothing depends on timing.
                      Positions, charges and outputs stay float64. */
} obem_precision;

/* field_eval / field_eval_backward flags */
#define OBEM_TGT_IS_SRC 1u  /* targets are the sources (same arrays, n_tgt == n_src):
                               the j == i term is skipped (eq. (nbody))          */
#define OBEM_WANT_V 2u      /* also write the potential V (eq. (BEM2) + point charges) */

typedef struct obem_ctx obem_ctx;      /* device, stream, workspace                  */
typedef struct obem_meshh obem_meshh;  /* bound mesh: derived cell data, cached LU   */

/* Flat triangular cells (section 2.2).  Device arrays of length n_panels.
 * Vertices a, b, c are counter-clockwise about the cell normal
 * n = (b-a)x(c-a)/|(b-a)x(c-a)|, which points from medium 1 (eps_r1) to
 * medium 2 (eps_r2).  kind: 0 = electrode cell (ed, Dirichlet row, eq.
 * (BEMpot)), 1 = dielectric interface cell (dd, Neumann row, eq. (BEMfld)).
 * eps_r1 / eps_r2 are read for dd cells only and may be NULL if there are
 * none.  Degenerate (zero-area) cells are rejected. */
typedef struct {
  int64_t n_panels;
  const double *ax, *ay, *az, *bx, *by, *bz, *cx, *cy, *cz;
  const int8_t *kind;
  const double *eps_r1, *eps_r2;
} obem_mesh;

typedef struct {
  int32_t iterations;       /* refinement sweeps performed                      */
  double backward_error;    /* max_i |r_i| / (max_i sum_j |A_ij| * max|sigma| + max|b|) */
  double residual_inf;      /* max_i |b_i - (A sigma)_i|                         */
} obem_solve_info;

/* Create a context on HIP device `device`, launching on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  *out receives the
 * handle.  The context owns its workspace (grown on demand). */
obem_status obem_create(obem_ctx **out, int device, void *hip_stream);
obem_status obem_destroy(obem_ctx *ctx);
/* Message of the last error on this context (never NULL; static storage of
 * the context). */
const char *obem_last_error(const obem_ctx *ctx);
/* Physical constants used by the library (CODATA 2018), host array out[6]:
 * eps0, k_e = 1/(4 pi eps0), e, m_e, k_B, atomic mass unit.  No GPU work. */
void obem_constants(double *out);

/* Kernel timing.  While enabled, the main kernels of every call are bracketed
 * with HIP events on the context stream (names: "order", "panel", "pair",
 * "pair_reduce", "scatter", "assemble", "lu", "solve", "panel_bwd",
 * "pair_bwd", "push_mc", "recombine", "compact").  obem_profile_read
 * synchronises the stream, writes up to max_entries (name, total ms,
 * launches) triples into host arrays names[max_entries][32], ms[], launches[]
 * in first-seen order, stores the count in *n_out and clears the record. */
obem_status obem_profile_enable(obem_ctx *ctx, int enable);
obem_status obem_profile_read(obem_ctx *ctx, int max_entries, char *names, double *ms, int64_t *launches,
                              int *n_out);
/* Work done by the forward pairwise kernels (eq. (nbody)) while profiling
 * was enabled, since the last call: host outputs *directed = (target,
 * source) terms evaluated by the directed kernel (targets and sources of the
 * tile pairs it takes, the zero self terms included) and *once = unordered
 * pairs evaluated once for both particles by the pair-once kernel (the pairs
 * of the tile pairs it does not leave to the directed kernel).  Together
 * they cover every pair: n (n - 1) interactions = (*directed - n) + 2 *once
 * for one field evaluation of n particles with targets = sources.
 * Synchronises the stream; either pointer may be NULL.  Resets the counts. */
obem_status obem_profile_work(obem_ctx *ctx, int64_t *directed, int64_t *once);

/* Bind a mesh: copies the cell data into the handle and derives normals,
 * areas, centroids, diameters and the far-field quadrature points.  The
 * collocation matrix is assembled lazily by the first bem_solve_charges. */
obem_status obem_mesh_bind(obem_ctx *ctx, const obem_mesh *mesh, obem_meshh **out);
obem_status obem_mesh_release(obem_ctx *ctx, obem_meshh *mesh);
/* Derived data of a bound mesh, copied into caller device arrays of length
 * n_panels (any may be NULL): area, centroid (3 arrays), diameter (longest
 * edge). */
obem_status obem_mesh_geometry(obem_ctx *ctx, const obem_meshh *mesh, double *area, double *cx,
                               double *cy, double *cz, double *diameter);

/* Collocation solve, eq. (matrixBEM): finds sigma with A sigma = rhs, where
 *   ed row i: A_ij = k_e * int_{C_j} dS'/|r_i - r'|                 (eq. (BEMpot))
 *   dd row i: A_ii = (eps_r1 + eps_r2)/2,
 *             A_ij = (eps_r2 - eps_r1)/(4 pi) n_i . int_{C_j} (r_i - r')/|r_i - r'|^3 dS'
 *                                                                   (eq. (BEMfld))
 * r_i = centroid of cell i; rhs = [V_i for ed rows ; sigma_F,i for dd rows].
 * The first call on a mesh assembles A (FP64, analytic integrals) and
 * factors it (LU with partial pivoting); later calls reuse the factors (the
 * paper reuses its inverse the same way).  Each call solves, then applies up
 * to max_refine refinement sweeps (residual with compensated FP64 dot
 * products, correction solved with the same factors) until the backward
 * error stops decreasing.  rhs and sigma_out are device arrays of length
 * n_panels (they may alias).  info (host) may be NULL: then nothing is
 * synchronised.  A zero pivot, or a smallest pivot below n * 2^-52 times the
 * largest (duplicate or coincident cells), gives OBEM_ESINGULAR.  Backward error above 1e-14
 * after the sweeps: OBEM_ENOCONV (sigma_out is still written, info filled). */
obem_status bem_solve_charges(obem_ctx *ctx, obem_meshh *mesh, const double *rhs, double *sigma_out,
                              int max_refine, obem_solve_info *info);

/* Adjoint of the collocation solve (not in the paper): g_rhs = A^{-T} g_sigma,
 * the gradient of a loss L(sigma) with respect to the left-hand side of eq.
 * (matrixBEM) given dL/dsigma: g_rhs_i = dL/dV_i on ed rows (sum over an
 * electrode's cells for dL/dV_electrode) and dL/dsigma_F,i on dd rows.  Uses
 * the cached inverse (assembling and factoring first if needed) and refines
 * against A^T with compensated residuals.  Arguments and errors as for
 * bem_solve_charges; the backward error in info refers to A^T. */
obem_status bem_solve_charges_adjoint(obem_ctx *ctx, obem_meshh *mesh, const double *g_sigma, double *g_rhs,
                                      int max_refine, obem_solve_info *info);

/* Influence of point charges on the collocation equations, section 3.3.2
 * (eqs. (potpart), (fldpart), (BEMpotpart), (BEMfldpart)): the charges'
 * potential and field averaged over each cell,
 *   Vbar_i = k_e/A_i sum_p q_p int_{C_i} dS/|r - x_p|
 *   Ebar_i = k_e/A_i sum_p q_p int_{C_i} (r - x_p)/|r - x_p|^3 dS
 * move to the left-hand side of eq. (matrixBEM):
 *   rhs_out_i = rhs_i - Vbar_i                                  (ed rows)
 *   rhs_out_i = rhs_i - eps0 (eps_r2 - eps_r1) Ebar_i . n_i     (dd rows)
 * so that bem_solve_charges(rhs_out) gives the cell charges in the presence
 * of the space charge.  sx, sy, sz, sq (charges in C): n_src device entries
 * (n_src may be 0: rhs_out = rhs).  rhs, rhs_out: n_panels device entries
 * (they may alias).  vbar and ebar_x/y/z (n_panels device entries each) are
 * optional outputs, NULL to skip; the three ebar arrays are given together
 * or not at all.  precision as for field_eval (cell/charge pairs within 3
 * cell diameters are always FP64 closed forms).  A charge exactly in a
 * cell's plane inside the cell contributes the principal value of the normal
 * field (0).  Sums are deterministic. */
obem_status bem_influence(obem_ctx *ctx, const obem_meshh *mesh, int64_t n_src, const double *sx,
                          const double *sy, const double *sz, const double *sq, const double *rhs,
                          double *rhs_out, obem_precision precision, double *vbar, double *ebar_x,
                          double *ebar_y, double *ebar_z);

/* Field at targets, eqs. (BEM3) and (nbody):
 *   E(x_t) = k_e sum_k sigma_k int_{C_k} (x_t - r')/|x_t - r'|^3 dS'
 *          + k_e sum_s q_s (x_t - x_s) / (|x_t - x_s|^2 + soft^2)^{3/2}
 * and with OBEM_WANT_V the potential (eq. (BEM2) and its point-charge
 * counterpart k_e q_s / (|d|^2 + soft^2)^{1/2}).  mesh may be NULL (no
 * cells; sigma ignored); n_src may be 0.  Source arrays sx, sy, sz, sq
 * (charges in C) have n_src entries, target arrays n_tgt; outputs Ex, Ey, Ez
 * (and V if requested, else V may be NULL) have n_tgt entries and are
 * overwritten.  A target exactly in a cell's plane inside the cell gets the
 * principal value of that cell's normal field (0).  soft >= 0 is the Plummer
 * softening length; with soft == 0 coincident distinct points are the
 * caller's responsibility (their term is dropped).
 * With OBEM_TGT_IS_SRC, OBEM_MIXED, soft > 0, no potential and 4097 to 2^24
 * charges, the pairwise sum evaluates every unordered pair of charges in
 * different 2048-charge blocks once for both (the pair term is
 * antisymmetric); its FP32 partial sums take up to 1920 n bytes of context
 * workspace per launch of up to 80 block distances, twice that when the
 * distances take more than one launch (15.4 GB at n = 4M), its tile-pair mask
 * (n / 256)^2 / 8 bytes, and the partial sums are added in FP64 in a fixed
 * order.  With more than one launch, a second stream of the context (default
 * priority, created on first use) adds each launch's partial sums while the
 * next launch runs; the caller's stream waits for it before the call
 * returns, so the call stays ordered on the caller's stream.
 * track_step uses the same evaluation for its field. */
obem_status field_eval(obem_ctx *ctx, const obem_meshh *mesh, const double *sigma, int64_t n_src,
                       const double *sx, const double *sy, const double *sz, const double *sq,
                       int64_t n_tgt, const double *tx, const double *ty, const double *tz, double soft,
                       obem_precision precision, unsigned flags, double *Ex, double *Ey, double *Ez,
                       double *V);

/* field_eval without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and error behaviour as
 * field_eval, but at most OBEM_NOALLOC_MAX_POINTS targets and sources
 * (larger counts: OBEM_EINVAL before any launch), and the workspace comes
 * from one static device array of OBEM_NOALLOC_SCRATCH_BYTES that the
 * library holds on each device it runs on until the process ends; no
 * hipMalloc, hipFree or allocating library call is made (OBEM_ENOMEM with a
 * message if a call ever needed more than the array).  Every call on one
 * device shares that device's array: calls that overlap on one GPU (other
 * contexts, other streams, other host threads) race and must be ordered by
 * the caller.  The kernels write every workspace entry they read, so the
 * array's contents left by an earlier call do not matter.  Kernel timing is
 * off during the call. */
#define OBEM_NOALLOC_MAX_POINTS 16384
#define OBEM_NOALLOC_SCRATCH_BYTES (80ull << 20)
obem_status field_eval_noalloc(obem_ctx *ctx, const obem_meshh *mesh, const double *sigma, int64_t n_src,
                               const double *sx, const double *sy, const double *sz, const double *sq,
                               int64_t n_tgt, const double *tx, const double *ty, const double *tz, double soft,
                               obem_precision precision, unsigned flags, double *Ex, double *Ey, double *Ez,
                               double *V);

/* Adjoint of field_eval for L = sum_t gE_t . E(x_t) (not in the paper):
 *   g_sigma_k = k_e sum_t gE_t . int_{C_k} (x_t - r')/|x_t - r'|^3 dS'
 *   g_t       = (dE(x_t)/dx_t)^T gE_t        (cells and point charges)
 *   g_s       = source-position part of the pairwise term
 * With OBEM_TGT_IS_SRC both position parts are summed into g_tx/g_ty/g_tz
 * and g_sx/g_sy/g_sz are ignored.  Any output may be NULL (not computed);
 * outputs are overwritten.  Sums are deterministic (fixed-order reductions,
 * no floating-point atomics); source tiles are recomputed, nothing is kept
 * from the forward call.  With OBEM_TGT_IS_SRC under the conditions of
 * field_eval's pair-once evaluation, the pairwise term J(d) a of each pair
 * of charges in different 1024-charge blocks is evaluated once for both
 * (partial sums and the second stream as in field_eval). */
obem_status field_eval_backward(obem_ctx *ctx, const obem_meshh *mesh, const double *sigma,
                                int64_t n_src, const double *sx, const double *sy, const double *sz,
                                const double *sq, int64_t n_tgt, const double *tx, const double *ty,
                                const double *tz, double soft, obem_precision precision, unsigned flags,
                                const double *gEx, const double *gEy, const double *gEz, double *g_sigma,
                                double *g_tx, double *g_ty, double *g_tz, double *g_sx, double *g_sy,
                                double *g_sz);

/* ---------------------------------------------------------------------------
 * Static field option (section 3.3.1) and signal induction (section 3.5)
 * ------------------------------------------------------------------------- */

/* Field of the cells on a uniform 3D grid: nodes lo + (i h0, j h1, k h2),
 * 0 <= i < nx etc. (each >= 2, nx*ny*nz < 2^31), values in caller-owned
 * device arrays ex, ey, ez of nx*ny*nz doubles, index (k*ny + j)*nx + i. */
typedef struct {
  int32_t nx, ny, nz;
  double lo[3];
  double h[3];    /* node spacing, > 0 */
  double *ex, *ey, *ez;
} obem_field_map;

/* Fill map->ex/ey/ez with the cell field of sigma (eq. (BEM3)) at the grid
 * nodes, computed once before tracking (the static option: it leaves out
 * the influence of the particles and the charging-up).  A node exactly in a
 * cell's plane inside the cell gets the principal value of that cell's
 * normal field. */
obem_status field_map_build(obem_ctx *ctx, const obem_meshh *mesh, const double *sigma,
                            const obem_field_map *map, obem_precision precision);

/* Trilinear interpolation of the map at n points (device SoA x, y, z);
 * points outside the grid box take the value at the nearest point of the
 * box.  Outputs Ex, Ey, Ez (n device doubles) are overwritten. */
obem_status field_map_eval(obem_ctx *ctx, const obem_field_map *map, int64_t n, const double *x,
                           const double *y, const double *z, double *Ex, double *Ey, double *Ez);

/* Shockley-Ramo current induced on one read-out electrode, eq. (ramo):
 *   i_s = sum over particles p of species s of q_p v_p . E_w(x_p),
 * with E_w the electrode's weighting field: either the cell field of sigma_w
 * (mesh and sigma_w given, map NULL; sigma_w = bem_solve_charges with that
 * electrode's cells at 1 V, every other ed cell at 0 V and no free charge on
 * dd cells -- the dynamic option) or a map of it (map given, mesh and sigma_w
 * NULL -- the static option).  Particles: n entries of device SoA positions,
 * velocities and species (charge -e for electrons (0) and anions (2), +e
 * for cations (1)).  current (host, 3 doubles, A): the sums for electrons,
 * cations and anions; requesting it synchronises the stream.  terms (device,
 * n doubles, may be NULL): the per-particle q v . E_w.  The sums are taken
 * in a fixed order (deterministic). */
obem_status induced_current(obem_ctx *ctx, const obem_meshh *mesh, const double *sigma_w,
                            const obem_field_map *map, int64_t n, const double *x, const double *y,
                            const double *z, const double *vx, const double *vy, const double *vz,
                            const int8_t *species, obem_precision precision, double *current,
                            double *terms);

/* ---------------------------------------------------------------------------
 * Transport step (sections 3.3-3.4)
 * ------------------------------------------------------------------------- */
#define OBEM_ELECTRON 0
#define OBEM_CATION 1
#define OBEM_ANION 2

/* Particle state: device arrays of length `capacity`, entries [0, n_live)
 * valid and ordered by increasing id.  Charge and mass follow from species
 * (electron -e, m_e; cation +e, gas.m_cation; anion -e, gas.m_anion).
 * n_live and next_id are host values updated by track_step. */
typedef struct {
  int64_t capacity;
  int64_t n_live;
  int64_t next_id;
  double *x, *y, *z, *vx, *vy, *vz;
  int8_t *species;
  int64_t *id;
} obem_particles;

/* Gas (section 3.4): electron cross sections xs (device, [5][n_nodes], m^2)
 * on nodes log-spaced from e_min to e_max (eV), interpolated linearly in the
 * normalised lethargy of eq. (leth) and clamped outside; process order
 * elastic, excitation 1, excitation 2, ionisation, attachment with
 * thresholds thr (eV; thr[3] is the ionisation energy).  Ions collide with
 * constant isotropic and backscattering cross sections. */
typedef struct {
  int32_t n_nodes;
  double e_min, e_max;
  const double *xs;
  double thr[5];
  double density;       /* gas number density, m^-3 */
  double temperature;   /* K */
  double m_gas, m_cation, m_anion;  /* kg */
  double ion_xs_iso, ion_xs_back;   /* m^2 */
  const double *xi;     /* device [n_nodes] or NULL: anisotropy xi(E) of the elastic
                           angle, eq. (anisotrop), cos theta = 1 - 2R(1 - xi)/(1 +
                           xi(1 - 2R)) about the incident direction; NULL =
                           isotropic */
  double penning_prob;  /* Penning transfer (section 3.4.4): an excitation whose
                           threshold is >= penning_level ionises the quencher with
                           this probability (0 = off); the electron takes the
                           excess energy, the cation a thermal speed */
  double penning_level; /* eV, ionisation potential of the quenching species */
} obem_gas;

/* Transport schemes (sections 3.3.5, 3.4.2). */
#define OBEM_NULL_COLLISION 0 /* constant-field flights with null collisions      */
#define OBEM_EULER 1          /* one flight in the start field, then the per-step
                                 collision test                                   */
#define OBEM_PEFRL 2          /* PEFRL (4 field evaluations at the intermediate
                                 positions, from the set-up and the charges still
                                 in the step), then the per-step collision test  */

typedef struct {
  double dt;            /* step length, s                                          */
  uint32_t step;        /* step counter (random stream coordinate)                 */
  uint64_t seed;        /* Philox key                                              */
  int32_t max_coll;     /* flights with a collision test per particle per step     */
  int32_t max_ion_per_step;  /* ionisations with children per particle per step   */
  double ion_v_cap;     /* speed bound for the ion null-collision rate, m/s        */
  double box_lo[3], box_hi[3];  /* world box; leaving it removes the particle      */
  double soft;          /* softening of the pairwise field                         */
  double r_rec;         /* recombination radius (eq. (distRecomb) as a parameter)  */
  obem_precision precision;
  int32_t resolve;      /* 1: rebuild the RHS from rhs0 + charging counts and
                           re-solve sigma before the field evaluation; 2: the
                           same, but when the RHS equals, bit for bit, the one
                           of the mesh's previous re-solve (no new charge, no
                           influence, same rhs0) that solve's sigma is copied
                           instead of solving again (the result is identical);
                           3: as 2, and when at most 4096 RHS entries changed
                           since that re-solve, sigma moves by the inverse's
                           columns of those entries times their change (sigma
                           agrees with a full re-solve to rounding; after 64
                           such updates the next change takes a full re-solve) */
  int32_t influence;    /* with resolve: also move the live particles' influence
                           onto the RHS before the solve (as bem_influence)       */
  const double *rhs0;   /* device, n_panels: [V_i ; sigma_F0,i]                    */
  int32_t stepper;      /* OBEM_NULL_COLLISION, OBEM_EULER or OBEM_PEFRL. Per-step
                           collision test: probability 1 - exp(-nu_tot dt) with
                           nu_tot = N sigma_tot(E) v at the end of the drift, the
                           process chosen in proportion to nu_k; at most one
                           collision per particle and step                      */
  const obem_field_map *map;  /* static option (section 3.3.1): if not NULL the field
                           of the set-up is interpolated in this map instead of
                           summed over the cells (resolve must then be 0); the
                           mesh, if given, still absorbs particles and collects
                           charging counts                                       */
  double *field_out;    /* device, 3 x n_live or NULL: the field at the start
                           positions (all Ex, then Ey, then Ez; particles in the
                           order of the state at the call)                      */
} obem_step_params;

typedef struct {
  int64_t n_live;
  int64_t recombined, absorbed, left_world, children, children_dropped;
  int64_t real_collisions[5];   /* electron processes, in table order           */
  int64_t null_collisions, ion_collisions, rate_overflow, flight_cap;
  int64_t dd_charge_deposited;  /* elementary charges landed on dd cells         */
  int64_t penning;              /* Penning transfers (pairs created)            */
} obem_step_stats;

/* One tracking step (ordered as in the paper's dynamic option):
 *  1. if p->resolve: rhs = rhs0 + e * dd_counts / area on dd rows
 *     (eq. (charge-up)), sigma = bem_solve_charges(rhs) with one
 *     refinement sweep (with resolve = 2
 *     skipped when rhs is unchanged since the mesh's last re-solve, with
 *     resolve = 3 also updated from the inverse when few entries changed);
 *  2. E at every live particle from the cells and all other particles,
 *     and each particle's nearest opposite-species partner;
 *  3. electron-cation pairs closer than r_rec recombine (eq. (distRecomb)):
 *     each electron proposes to its nearest cation, each cation accepts its
 *     nearest proposer (ties: lower id);
 *  4. constant-field flights over dt with null-collision Monte Carlo
 *     (Philox4x32-10 keyed by seed, counter (id, step, flight)); ionisation
 *     creates an electron and a cation (eq. (distIoni)); attachment turns the
 *     electron into an anion; a flight chord crossing a cell absorbs the
 *     particle (dd hits add the particle charge to dd_counts);
 *  5. survivors are compacted in id order and children appended with ids
 *     next_id, next_id + 1, ...
 * dd_counts: device int64 [n_panels] (only dd entries change).  sigma:
 * device [n_panels], read (and rewritten when p->resolve).  The call
 * synchronises the stream (the new n_live is needed on the host); stats
 * (host) may be NULL.  Children beyond capacity are dropped and counted:
 * OBEM_ECAPACITY after the step completes. */
obem_status track_step(obem_ctx *ctx, obem_meshh *mesh, obem_particles *state, const obem_gas *gas,
                       const obem_step_params *p, int64_t *dd_counts, double *sigma,
                       obem_step_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* OBEM_H */
