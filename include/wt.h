/*
 * wt.h -- C ABI of the MI355X (gfx950) adaptive wavelet TRiSK shallow-water library.
 *
 * Method: Aechtner, Kevlahan & Dubos, "A conservative adaptive wavelet method for the
 * shallow water equations on the sphere" (arXiv:1404.0405).  Section, equation and table
 * numbers below refer to that paper.
 *
 * Conventions shared by every call
 *   - Every int-returning call returns WT_OK (0) or a negative WT_E* code; the message of the
 *     last failure on the calling thread is returned by wt_last_error().
 *   - Pointer arguments named *host* are caller-owned host memory, read or written during the
 *     call only; the library keeps no pointer.  Device pointers are named *_device.
 *   - Level j runs over jmin..jmax.  Level j has n = 2^j, N = 10 n^2 + 2 nodes,
 *     E = 30 n^2 edges and T = 20 n^2 triangles (Table 1).
 *   - Canonical ordering (the only layout exchanged at this boundary; device layouts are
 *     internal): node (L,i,j) with lozenge 0 <= L < 10 and 0 <= i,j < n has id
 *     (L*n + i)*n + j; the north and south poles are 10n^2 and 10n^2+1.  Lozenges 0..4 are
 *     the faces (U_k, L_k, U_k+1) + (U_k, U_k+1, N), lozenges 5..9 the faces
 *     (L_k, S, L_k+1) + (L_k, L_k+1, U_k+1) of the icosahedron with upper ring U_k at
 *     longitude 72k and lower ring L_k at 72k+36 degrees; i runs from corner c00 to c10, j
 *     from c00 to c01.  Edge 3*id + d joins node (i,j) to (i+1,j), (i+1,j+1), (i,j+1) for
 *     d = 0,1,2; the normal velocity u_e is positive from the owning node to the other end.
 *     Level j+1 node (L,2i,2j) is level j node (L,i,j) (nested grids, Sec. 2.1-2.2).
 *   - Prognostic variables: dh = h - H at nodes (metres) and u at edges (m/s), point values.
 *   - A wt_grid is used by one host thread at a time; all device work of a grid is ordered on
 *     its stream.
 */
#ifndef WT_H
#define WT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wt_grid wt_grid;

enum {
  WT_OK = 0,
  WT_EINVAL = -1,   /* bad argument (level, size, null pointer, parameter range) */
  WT_ENOMEM = -2,   /* host or device allocation failed */
  WT_EDEVICE = -3,  /* HIP runtime error, or no gfx950 device */
  WT_ESTATE = -4,   /* call out of order (e.g. wt_step before wt_set_state) */
  WT_ENUMERIC = -5  /* non-finite value found in the state */
};

/* Time schemes (Sec. 3.1): the paper's four-stage third-order SSP Runge-Kutta, and classical
 * four-stage RK4.  Both evaluate the tendencies four times per step. */
enum { WT_RK4 = 0, WT_SSPRK43 = 1 };

/* Arithmetic of the tendencies and transforms.  WT_FP64: everything in double.
 * WT_FP32_TENDENCY: single precision for the TRiSK quantities q, K, B, qF^perp and the velocity
 * products of the tendencies, and for the stencil sums of the velocity transform's predictions
 * (Sec. 4.1: 18 coarse edges per half-edge pair, 9 per interior edge) in the forward transform
 * (details), the inverse transform and the prolongation of inactive points.  Double precision is
 * kept for the prognostic state and the Runge-Kutta accumulation, the mass flux F, its
 * divergence and its restriction R_F, the combination of each prediction with the stored values
 * (detail = value - prediction, value = detail + prediction), the whole height transform (its
 * prediction, eq. (WTpred), is part of the area-weighted restriction R_h, eq. (Rh), whose exact
 * inversion by the adapt's reconstruction keeps the partial transform mass-conservative), and the
 * mass/energy diagnostics (the paper keeps the quantities that carry the mimetic properties in
 * double and truncation-limited ones in single, Sec. 5.1), so mass is conserved to round-off in
 * both modes. */
enum { WT_FP64 = 0, WT_FP32_TENDENCY = 1 };

/* Equations.  WT_SWE: the rotating shallow-water equations (height) and (velo) of Sec. 3.1.
 * WT_ADVECTION: the height equation alone, its thickness flux h u carried by the velocity field
 * of the state, which stays fixed (du/dt = 0; the advection test of Sec. 6.1). */
enum { WT_SWE = 0, WT_ADVECTION = 1 };

/* Thresholds of the adapt (Sec. 3.1).  WT_THR_RELATIVE: eps_h = eps max|dh|, eps_u = eps max|u|
 * over the active points.  WT_THR_QG / WT_THR_IG: the regime thresholds of Sec. 3.1 from the
 * typical velocity U, length L and Coriolis parameter f of the flow (scale_u, scale_l, scale_f)
 * and the gravity-wave speed c = sqrt(g H).  The printed formulas give the velocity threshold in
 * m/s and the height threshold in geopotential units (m^2/s^2) with their two names exchanged;
 * read with the names swapped back and the height threshold divided by g:
 *   quasi-geostrophic (Ro = U / (f L)):  eps_u = U Ro eps^(3/2),  eps_h = f U L Ro eps^(3/2) / g,
 *   inertia-gravity:                     eps_u = U eps^(3/2),     eps_h = c U eps^(3/2) / g. */
enum { WT_THR_RELATIVE = 0, WT_THR_QG = 1, WT_THR_IG = 2 };

typedef struct {
  double radius;      /* sphere radius a [m], default 6.371e6 */
  double omega;       /* rotation rate [1/s], default 7.292e-5 (Sec. 6) */
  double gravity;     /* g [m/s^2], default 9.80616 (Sec. 6) */
  double mean_depth;  /* H [m], h = H + dh; default 2.94e4 / g; > 0 (>= 0 for WT_ADVECTION) */
  int rk;             /* WT_RK4 (default) or WT_SSPRK43 */
  int precision;      /* WT_FP64 (default) or WT_FP32_TENDENCY */
  double viscosity;   /* nu [m^2/s] >= 0, default 0: the dissipative form of Sec. 3.1 adds
                         nu div grad dh to the height and nu (grad div u - grad^perp curl u) to
                         the velocity tendency */
  int equations;      /* WT_SWE (default) or WT_ADVECTION */
  int threshold;      /* WT_THR_RELATIVE (default), WT_THR_QG or WT_THR_IG */
  double scale_u;     /* U [m/s] of the regime thresholds (> 0 when they are used) */
  double scale_l;     /* L [m] of the quasi-geostrophic thresholds */
  double scale_f;     /* f [1/s] of the quasi-geostrophic thresholds */
} wt_params;

typedef struct {
  double mass;        /* sum_k A_k (H + dh_k) on level jmin [m^3] (Sec. 4.1); below jmax A_k
                         are the effective areas of the height transform */
  double mass_reconstructed; /* the same sum of the jmax reconstruction (equal up to rounding) */
  double energy;      /* E of Sec. 7.2 of the jmax reconstruction [m^5/s^2] */
  double max_abs_dh;  /* max |dh| over active nodes of all levels */
  double max_abs_u;   /* max |u| over active edges of all levels */
  int64_t active_nodes[16]; /* per level j (index j), active node count */
  int64_t active_edges[16]; /* per level j (index j), active edge count */
  int32_t finest_level; /* highest level holding an active point: the maximum level the
                           thresholds select (Sec. 3.1: Jmax set implicitly by eps, the grid's
                           jmax acting as a cap) */
  int32_t pad_;
} wt_diag;

/* Create a grid with levels jmin..jmax (0 <= jmin <= jmax <= 12) and adaptivity patch size
 * patch in {4, 8, 16} (Sec. 5.2: patches are the smallest unit of the adapted structure;
 * results do not depend on it).  Builds the geometry of every level on the host (Sec. 4.1)
 * and uploads it; selects HIP device 0 unless one is current.  Returns NULL on error.
 * The geometry-only host tables of each level and level pair (those not depending on the
 * effective areas, Sec. 4.1) are kept in a process-wide cache and shared by later grids. */
wt_grid* wt_grid_create(int jmin, int jmax, int patch);
/* Frees the host table cache of wt_grid_create (existing grids are not affected). */
void wt_table_cache_clear(void);

/* Frees all host and device memory of the grid.  NULL is accepted. */
void wt_grid_destroy(wt_grid* g);

/* Set / read the physical and numerical parameters.  wt_set_params before wt_set_state;
 * radius and omega are fixed when the grid is created (they shape the geometry), so a
 * different radius/omega returns WT_EINVAL. */
int wt_set_params(wt_grid* g, const wt_params* p);
int wt_get_params(const wt_grid* g, wt_params* p);

/* Sizes of level `level`: nodes, edges, triangles.  Any pointer may be NULL. */
int wt_grid_info(const wt_grid* g, int level, int64_t* n_nodes, int64_t* n_edges,
                 int64_t* n_tris);

/* Unit-sphere coordinates of level `level`, canonical order, host arrays:
 * node_xyz_host[3N], edge_mid_xyz_host[3E] (arc midpoint), edge_tangent_xyz_host[3E] (unit
 * tangent at the midpoint, pointing along positive u).  Any pointer may be NULL. */
int wt_grid_coords(const wt_grid* g, int level, double* node_xyz_host,
                   double* edge_mid_xyz_host, double* edge_tangent_xyz_host);

/* Load the prognostic state of level `level` from host arrays dh_host[N], u_host[E]
 * (canonical order).  Levels jmin..level become fully active, the coarser ones computed by the
 * forward transform (height restriction eq. (Rh), velocity restriction by half-edge means);
 * levels above `level` become inactive.  On a uniform grid (jmin == jmax) this is the whole
 * state. */
int wt_set_state(wt_grid* g, int level, const double* dh_host, const double* u_host);

/* Same, from device arrays (stream-ordered on the grid's stream). */
int wt_set_state_device(wt_grid* g, int level, const void* dh_device, const void* u_device);

/* Read the state of level `level` into host arrays dh_host[N], u_host[E] (canonical
 * order): on a multilevel grid the level is reconstructed by the inverse transform from jmin
 * with the details of the active points (zero elsewhere), so its mass equals the mass on jmin.
 * node_active_host[N] / edge_active_host[E] receive 1 for active points.  Any pointer may be
 * NULL.  Synchronises the grid's stream. */
int wt_get_state(wt_grid* g, int level, double* dh_host, double* u_host,
                 uint8_t* node_active_host, uint8_t* edge_active_host);

/* Advance the state by one Runge-Kutta step of length dt seconds (four tendency
 * evaluations, eqs. (height) and (velo), TRiSK discretisation with the energy-conserving
 * qF^perp, Sec. 3.1).  On a multilevel grid every stage (Sec. 3.1, time step) fills inactive
 * points by zero-detail prediction, computes q, K, B, F and qF^perp on every level, restricts
 * F (flux restriction R_F, eqs. (restr_flux), (ho_flux), (kml)), qF^perp (half-edge mean) and
 * B (injection) to coarser levels at non-leaf points, and updates the active points of every
 * level; after the step the coarse heights at complete nodes are replaced by the height
 * restriction of the finer level (partial transform, height only).  No adaptation.
 * Asynchronous on the grid's stream. */
int wt_step(wt_grid* g, double dt);

/* Adapt the grid (Sec. 2.3, 3.1): wavelet details of all levels; thresholds
 * eps_h = eps max|dh|, eps_u = eps max|u| over active points; significant iff |d| >= eps_var;
 * adjacent zone (same-level neighbours and next-level children of significant points); all of
 * jmin; h/u consistency and the coarse prediction stencils of every active point; then the
 * inverse transform rewrites every active fine point from its coarse level and the kept
 * details.  Coarse values and the mass on jmin are unchanged.  eps = 0 keeps every point.
 * No-op on a uniform grid.  Synchronises. */
int wt_adapt(wt_grid* g, double eps);

/* Forward transform: compute and keep the wavelet details of every level pair (eqs. (WTpred)
 * for height, the velocity prediction of Sec. 4.1) from the current state.  Read them with
 * wt_get_details.  No-op on a uniform grid. */
int wt_forward(wt_grid* g);

/* Inverse transform: rewrite every fine level from jmin with the details of the active
 * points, making all levels consistent (R_h of each level is the level below).  No-op on a
 * uniform grid. */
int wt_inverse(wt_grid* g);

/* Details computed by the last wt_forward / wt_adapt for the pair (level-1, level), coarse
 * canonical order of level-1: dh_host[E_c] height detail of the midpoint node of each coarse
 * edge, dpair_host[E_c] velocity detail of each pair of half-edges, dint_host[3 T_c] velocity
 * details of the three fine edges inside each coarse triangle.  Test hook; synchronises. */
int wt_get_details(wt_grid* g, int level, double* dh_host, double* dpair_host, double* dint_host);

/* The adaptive stage runs over work lists: after every change of the masks the library builds,
 * per level, the rings of the active points (3 rings: where q_v, F, B, q_e, Q and the fine
 * divergence are computed; 5 rings: where inactive points are prolonged) and compacts them into
 * index lists by wavefront ballot and prefix scan (Sec. 5.2 works on the active patches only).
 * enable = 0 runs every stage kernel over whole levels instead (test hook: the two agree
 * bitwise at every active point).  Default: enabled.  Synchronises. */
int wt_set_work_lists(wt_grid* g, int enable);

/* The listed step of a multilevel grid (Sec. 3.1 per stage: prolongation, intermediates,
 * restriction, tendencies; then the partial height transform) merges the launches of work that
 * does not depend on each other -- the same kernel on every level, the odd and interior
 * prolongation of a pair, the edge and B restriction of a pair -- into one launch each (88
 * launches per RK4 step for five levels instead of ~185).  enable = 0 launches one kernel per
 * level and kind (test hook: the two agree bitwise).  Default: enabled.  Synchronises. */
int wt_set_step_phases(wt_grid* g, int enable);

/* Dense finest level (Sec. 3.1 stage on the finest level, Sec. 4.1-4.3 restriction from it):
 * when the 3-ring support of the finest level's active points holds at least min_fraction of
 * its elements (always, when the stage runs over whole levels), the level's tile elements run
 * through the lattice kernel of the uniform stage in a masked form -- tendencies zero at
 * inactive points, and the mass flux F, qF^perp Q and the Bernoulli function B of every element
 * stored for the restriction chain; with work lists only the tiles of each lozenge that hold a
 * point of the 5-ring support -- and only the rim round the twelve lozenge corners through the
 * listed table-driven kernels.  When the level below the finest is 6 or more and its support
 * is as dense by the same measure, it computes its intermediates F, Q and B the same way, in an
 * intermediates-only form of the kernel (no tendency, no stage output; the level's tendencies
 * stay listed, after the restriction from the finest level has replaced F, Q and B at its
 * non-leaf points).  Results agree with the listed stage to round-off (the lattice kernel sums
 * in another order), not bitwise.  min_fraction > 1 turns it off (the default); enabling builds
 * the two levels' lattice geometry (finest level 6 or more, inviscid shallow-water form only:
 * other forms and ensemble steps keep the listed kernels).  WT_EINVAL for a negative or
 * non-finite fraction or a finest level below 6.  Synchronises. */
int wt_set_dense_levels(wt_grid* g, double min_fraction);
/* The level below the finest runs its intermediates through the lattice kernel only when its
 * lattice has at least min_tiles tile positions (the kernel runs one workgroup per position):
 * -1, the default, takes the device's compute-unit count, below which the listed kernels are
 * faster; 0 lets any size through (test hook for small grids).  WT_EINVAL below -1. */
int wt_set_dense_min_tiles(wt_grid* g, int min_tiles);

/* Replace the active masks of `level` (host arrays of N and E bytes, 1 = active).  Test hook,
 * used to resynchronise masks with a reference at exact threshold ties. */
int wt_set_mask(wt_grid* g, int level, const uint8_t* node_active_host, const uint8_t* edge_active_host);

/* Evaluate the tendencies d(dh)/dt and du/dt of the current state of a full level into host
 * arrays ddh_host[N], du_host[E] (canonical order).  Test and diagnostic hook; synchronises. */
int wt_tendency(wt_grid* g, int level, double* ddh_host, double* du_host);

/* Diagnostics of the current state (mass Sec. 4.1, energy Sec. 7.2, maxima); synchronises.
 * Returns WT_ENUMERIC (and fills the struct) if the state holds a non-finite value. */
int wt_diagnostics(wt_grid* g, wt_diag* d);

/* Stable time step dt = cfl * min(1/omega_max, min_e d_e/|u_e|) over the finest active
 * level, omega_max = max sqrt(f^2 + g h (pi/d_e)^2) (Sec. 3.1, with the wavenumber squared).
 * Returns a negative value on error. */
double wt_suggest_dt(wt_grid* g, double cfl);

/* Use `hip_stream` (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream) for all
 * later device work of the grid; NULL selects the library's own stream. */
int wt_set_stream(wt_grid* g, void* hip_stream);

/* Device allocator of the grid's buffers, e.g. PyTorch's caching allocator.  With g non-NULL,
 * later allocations of g (buffers created lazily: work lists, scratch, checkpoint staging ...)
 * use it; with g NULL it becomes the allocator of every grid created afterwards, so that all of
 * their device buffers come from it.  alloc(bytes, ctx) returns device memory of the current
 * HIP device (NULL on failure: the calling function then fails with WT_EDEVICE); free_(ptr,
 * ctx) returns it.  The library waits for all queued device work before each free_, so the
 * allocator may hand the memory out again at once.  Buffers keep the allocator that produced
 * them.  Both functions NULL: hipMalloc / hipFree (the default).  WT_EINVAL if only one is
 * given.  The pair (and ctx) must stay valid while a buffer they produced is alive. */
int wt_set_allocator(wt_grid* g, void* (*alloc)(size_t bytes, void* ctx), void (*free_)(void* ptr, void* ctx),
                     void* ctx);

/* Live device buffers owned by grid g: count and bytes from an allocator hook (n_hook,
 * bytes_hook) and from hipMalloc (n_direct, bytes_direct).  Any pointer may be NULL. */
int wt_alloc_stats(const wt_grid* g, int64_t* n_hook, int64_t* bytes_hook, int64_t* n_direct,
                   int64_t* bytes_direct);

/* Kernel timing for measurement: when enabled, every launch of the uniform-level TRiSK stage
 * kernels and of the masked lattice kernel is bracketed by HIP events on the grid's stream.  wt_kernel_time returns the summed
 * device time (ms), the launch count and the summed algorithmic bytes of the kernel named
 * `name` since the last reset (total_bytes may be NULL).  Algorithmic bytes count every table
 * entry, input and output element of a launch once: table-driven kernels per triangle 96 B +
 * q_v, per element 176 B + 6 intermediates (edge_cell) and 504 B + 4 intermediates + the
 * stage's Runge-Kutta arrays (tend); the lattice kernel per element the stage input (32 B)
 * and the Runge-Kutta arrays, plus its shared geometry (464 B per tile position) once for the
 * 10 lozenges; its masked form on a dense finest level (trisk_lattice_masked) also the four mask
 * bytes and the stored F, Q and B; its intermediates-only form on the level below
 * (trisk_lattice_inter) the stage input, the geometry's share and the stored F, Q and B.  Names
 * are listed by wt_kernel_names (comma separated). */
int wt_timing_enable(wt_grid* g, int enable);
int wt_timing_reset(wt_grid* g);
int wt_kernel_time(wt_grid* g, const char* name, double* total_ms, int64_t* launches, double* total_bytes);
/* Units the last timed launch of kernel `name` processed: elements (a node and its three edges)
 * for trisk_edge_cell, trisk_tend, trisk_lattice, trisk_lattice_masked and trisk_lattice_inter
 * (the lattice kernel: its regular tiles of all ten lozenges, or the flagged ones), triangles for
 * trisk_vertex; 0 if none was timed. */
int wt_kernel_units(wt_grid* g, const char* name, int64_t* units);
const char* wt_kernel_names(void);

/* Host-only inspection of the grid builder (no device needed): builds level `level` with
 * the given radius [m] and omega [1/s] and copies selected tables into caller arrays, canonical
 * order; any pointer may be NULL.  A_i_host[N] cell areas, A_v_host[T] triangle areas,
 * d_e_host[E] node-node arc lengths, l_e_host[E] dual edge lengths, e_nodes_host[2E]
 * from/to node of every edge, ecp_host[10E] and w_host[10E] the perpendicular-flux stencil
 * and weights w_{e,e'} of the energy-conserving qF^perp (Sec. 3.1; padded slots hold e itself
 * with weight 0).  Sizes are those of wt_grid_info.  For tests of the builder. */
int wt_host_level_tables(int level, double radius, double omega, double* A_i_host,
                         double* A_v_host, double* d_e_host, double* l_e_host,
                         int32_t* e_nodes_host, int32_t* ecp_host, double* w_host);

/* Host-only inspection of the inter-scale tables between levels jc and jc+1 of a hierarchy
 * jc..jmax (no device needed; jc < jmax <= 8).  Coarse sizes Nc, Ec, Tc are those of level jc.
 * cells_host[4Ec]: for every coarse edge a->b its cells (a, b, p, q), p opposite in the left
 * and q in the right triangle; st_host[4Ec] prediction weights s~_cm = A_cm / A_m of the
 * height transform (eq. (WTpred), Sec. 4.1); s_upd_host[4Ec] update weights s_km = A_km / A_k
 * (eq. (WTupd)); A_c_host[Nc] effective coarse cell areas; v_sten_host[9Tc] the coarse edges of
 * each coarse triangle's velocity stencil; w_int_host[27Tc] prediction weights of its three
 * interior fine edges (Sec. 4.1); w_pl_host[9Ec], w_pr_host[9Ec] weights of (p1 - p2) on the
 * stencils of the left / right triangle; rf_f_host[3Ec], rf_fw_host[3Ec], rf_c_host[8Ec],
 * rf_cw_host[8Ec] the flux restriction (eqs. (restr_flux), (ho_flux), (kml)): integrated
 * coarse flux = sum rf_fw * (l F)[rf_f] + sum rf_cw * c[rf_c], fine edge / node ids.  Any
 * pointer may be NULL.  For tests of the builder. */
int wt_host_pair_tables(int jc, int jmax, double radius, double omega, int32_t* cells_host,
                        double* st_host, double* s_upd_host, double* A_c_host,
                        int32_t* v_sten_host, double* w_int_host, double* w_pl_host,
                        double* w_pr_host, int32_t* rf_f_host, double* rf_fw_host,
                        int32_t* rf_c_host, double* rf_cw_host);

/* Host-only check of the lattice form of the uniform stage for level `level` (6 <= level <= 9;
 * no device needed): builds the shared reference geometry of the lozenge lattice (all 10
 * lozenges are congruent under rotations of the icosahedron, Sec. 2.2), verifies the halo
 * addressing of every regular tile, and compares the reference geometry with the canonical
 * tables of every lozenge.  n_tiles: regular tiles per lozenge; n_rim: elements left to the
 * table-driven kernels; max_rel_err: largest relative difference of cell areas, edge lengths
 * and sorted perpendicular-flux weights (relative to the row's largest weight) between the
 * reference and every lozenge.  For tests. */
int wt_host_lattice_check(int level, int64_t* n_tiles, int64_t* n_rim, double* max_rel_err);

/* ---------------------------------------------------------------------------------------
 * Learned adjacent zone (an addition to the method, not from the paper).  The paper's adjacent
 * zone (Sec. 2.3) activates the next-level children of every significant point.  A small
 * network proposes instead, for every quadrant of every patch, whether those children are
 * needed; the exact threshold test after each step redoes the step with the blanket zone when
 * a dropped quadrant still holds a significant point.
 *
 * Network: 64 features -> 128 -> 128 (ReLU) -> 4 (sigmoid).  Parameters are one float vector
 * of WT_MLP_PARAMS values in the order W1 [64][128] (row-major, [input][output]), b1[128],
 * W2 [128][128], b2[128], W3 [128][4], b3[4].  Matrix products run on the matrix cores with
 * bfloat16 operands (rounded to nearest even: inputs, weights, hidden activations and, in the
 * backward pass, the errors) and FP32 accumulation; biases, the master weights, the optimiser
 * and the loss are FP32.  Loss: mean binary cross-entropy over samples and the 4 outputs.
 * Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).  Feature and label
 * arrays are device memory, row-major [n][64] and [n][4]. */
typedef struct wt_mlp wt_mlp;
enum { WT_MLP_INPUTS = 64, WT_MLP_OUTPUTS = 4, WT_MLP_PARAMS = 25348 };

/* Create a network with the given initial parameters (host array of WT_MLP_PARAMS floats;
 * the caller draws them).  Uses the current HIP device.  Returns NULL on error. */
wt_mlp* wt_mlp_create(const float* params_host);
void wt_mlp_destroy(wt_mlp* m);
/* Stream for the network's device work (NULL: the library's own stream). */
int wt_mlp_set_stream(wt_mlp* m, void* hip_stream);
/* Copy the current FP32 parameters to params_host[WT_MLP_PARAMS]; synchronises. */
int wt_mlp_get_params(wt_mlp* m, float* params_host);
/* p_device[n][4] = sigmoid(network(x_device[n][64])).  Asynchronous on the network's stream. */
int wt_mlp_forward(wt_mlp* m, const float* x_device, int64_t n, float* p_device);
/* Gradient of the loss on (x, y) with respect to the parameters into grad_host[WT_MLP_PARAMS]
 * (may be NULL) and the loss into *loss (may be NULL); no update.  Synchronises. */
int wt_mlp_gradient(wt_mlp* m, const float* x_device, const float* y_device, int64_t n,
                    float* grad_host, double* loss);
/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the gradient of wt_mlp_gradient, bitwise, without any
 * allocation and without synchronising.  grad_device[WT_MLP_PARAMS + 1] (device memory) receives
 * the gradient and, in its last entry, the loss summed over samples and outputs (the mean loss
 * is that / (4 n)).  At most 1024 samples per call (WT_EINVAL beyond).  The per-tile partial
 * sums live in a 6.6 MB scratch array that the library holds on every GPU it has run on until
 * the process ends; every call on a GPU uses that GPU's one array, so calls that overlap on one
 * GPU (on different streams or host threads) race and must be serialised by the caller.
 * Asynchronous on the network's stream. */
int wt_mlp_gradient_noalloc(wt_mlp* m, const float* x_device, const float* y_device, int64_t n,
                            float* grad_device);
/* One Adam step with learning rate lr on the batch (x, y); *loss (may be NULL) receives the
 * loss before the step, which synchronises; with loss NULL the call is asynchronous. */
int wt_mlp_train_step(wt_mlp* m, const float* x_device, const float* y_device, int64_t n, double lr,
                      double* loss);

/* Patches of the learned zone: at level j (jmin < j < jmax, j >= 3) the lattice of every
 * lozenge is cut into 8 x 8 element patches, patch (L, pi, pj) -> index (L m + pi) m + pj with
 * m = 2^j / 8; quadrant c = 2a + b of a patch holds the elements (8pi + 4a .. +3, 8pj + 4b .. +3),
 * whose next-level children form patch (L, 2pi + a, 2pj + b) of level j+1.  wt_patch_count
 * returns the number of patches of `level` (0 for levels without a gate, negative on error). */
int64_t wt_patch_count(const wt_grid* g, int level);
/* Features x_device[count][64] of every patch of `level`, from the wavelet details and
 * thresholds of the last wt_adapt (or of the last judged step) and the current masks: with
 * r = clamp(log2(|d| / eps_var), -16, 4) / 8 the size of a detail against its threshold,
 * [0..35] the largest r of level-j height, level-j velocity, level-(j+1) height and
 * level-(j+1) velocity details over the patch and its 8 lattice neighbours (9 each; a
 * neighbour outside the lozenge repeats the patch), [36..51] the same four per quadrant,
 * [52..55] the active fraction of each quadrant's child patch, [56..59] the fraction of
 * significant level-j points of each quadrant, [60] the active fraction of the patch's nodes,
 * [61] (j - jmin) / (jmax - jmin), [62] 1, [63] 0.  Synchronises. */
int wt_patch_features(wt_grid* g, int level, float* x_device);
/* Labels y_device[count][4]: 1 where the quadrant holds a significant level-j point of the
 * current significant set (the last wt_adapt, or the test after the last judged step) -- the
 * quadrants whose children the blanket zone activates.  Synchronises. */
int wt_patch_labels(wt_grid* g, int level, float* y_device);
/* Use network m (NULL: the paper's blanket zone) to gate the children rule of later wt_adapt
 * calls: a quadrant's significant points activate their children only where the network's
 * probability is >= threshold (threshold > 1 drops every quadrant).  The step after a gated
 * adapt is judged by the threshold test on the new state: if a quadrant whose children were
 * dropped holds a significant point, the state and masks from before that adapt are restored
 * and the adapt and step are redone with the blanket zone.  The grid keeps the pointer; the
 * caller keeps m alive while it is set. */
int wt_set_predictor(wt_grid* g, wt_mlp* m, double threshold);
/* Test hook of the threshold test: at the next gated wt_adapt, withhold the children rule from
 * all four quadrants of patch `patch` (index as above) of `level` whatever the network
 * proposes, so that the following step is judged with those quadrants dropped where they are
 * significant.  Needs a predictor (WT_ESTATE otherwise); WT_EINVAL for a level without patches
 * or a patch out of range.  Several calls add up; the list is cleared by the gated adapt. */
int wt_debug_force_drop(wt_grid* g, int level, int64_t patch);

/* Number of steps redone by the threshold test since the grid was created. */
int wt_redo_count(const wt_grid* g, int64_t* redo);

/* ---------------------------------------------------------------------------------------
 * Ensembles (an addition to the method, not from the paper): independent members -- grids of
 * any levels, thresholds and precision -- advanced together.  One step of the ensemble is ONE
 * launch of a HIP graph that holds every member's Runge-Kutta step: when every member is a
 * multilevel grid stepping over work lists, as one launch per phase of the step over all
 * members' work (prolongation, intermediates, restriction, tendencies, partial transform), else
 * each member's step on its own stream; the graph is captured again (or updated in place) only
 * when a member's work lists, parameters or time step changed since the last capture.  Adapt
 * runs member by member on a few host threads (it reads list counts back to the host).  With the
 * learned zone, each member's step is judged after the graph and redone on its own if needed. */
typedef struct wt_ensemble wt_ensemble;
/* members: n distinct grids with distinct streams (the caller keeps them alive). */
wt_ensemble* wt_ensemble_create(wt_grid* const* members, int n);
void wt_ensemble_destroy(wt_ensemble* e);
/* wt_adapt of every member with eps_host[k]. */
int wt_ensemble_adapt(wt_ensemble* e, const double* eps_host);
/* One step of every member with dt_host[k] as one graph launch (or, batched, one persistent
 * launch); synchronises. */
int wt_ensemble_step(wt_ensemble* e, const double* dt_host);
/* Number of graph captures (batched: step plans built) and launches so far. */
int wt_ensemble_stats(const wt_ensemble* e, int64_t* captures, int64_t* launches);
/* on != 0: later steps run batched -- ONE persistent cooperative launch covers every member's
 * whole multilevel step.  The step's phases (prolongation pair by pair upwards, intermediates,
 * restriction pair by pair downwards, tendencies, per stage; then the partial height transform)
 * follow one another with a grid-wide barrier; within a phase, the jobs of all members (one per
 * member, level or pair and kernel) are cut into chunks of consecutive work-list entries that the
 * workgroups take from a global work queue (an atomic counter per phase).  Every entry runs the
 * same per-point code as the unbatched step, so results are bitwise those of stepping the members
 * one by one.  The launch shape (workgroups per CU, entries per chunk, work queue or a fixed
 * round-robin deal of the chunks) is tuned on line: the first steps each try one candidate, timed
 * with events on the ensemble's stream, and the fastest is kept.  Every member must be multilevel (jmin < jmax); WT_EINVAL otherwise.  on = 0 returns to
 * the graph step. */
int wt_ensemble_set_batched(wt_ensemble* e, int on);
/* Launch shape in use (workgroups per CU, entries per chunk, *queue = 1: chunks from the work
 * queue, 0: dealt round-robin; zeros before the first batched step), whether tuning has finished
 * (*tuned = 1) and the device time of the last batched launch in ms.  Any pointer may be NULL. */
int wt_ensemble_tuning(const wt_ensemble* e, int* blocks_per_cu, int* chunk, int* queue, int* tuned,
                       float* last_ms);

/* Checkpoint / restart.  wt_save writes the grid's state to the file `path` (binary): levels,
 * patch size, parameters, the thresholds of the last adapt and the redo count, then per level
 * the raw state of every point (active or not) and the masks.  wt_load reads such a file into a
 * grid created with the same jmin, jmax and patch (and the same radius and rotation rate; the
 * other parameters are taken from the file), rebuilds the work lists and leaves the grid ready
 * to step: continuing from a loaded checkpoint gives bitwise the states of continuing the saved
 * run (a learned predictor is not part of the file; set it again).  Errors: WT_EINVAL for a
 * null argument, an unreadable or unwritable path, or a file that is not a checkpoint of this
 * grid's shape (the grid is then unchanged); WT_ESTATE for wt_save without a state;
 * WT_EDEVICE for a device failure. */
int wt_save(wt_grid* g, const char* path);
int wt_load(wt_grid* g, const char* path);

/* Thread-local message of the last failing call ("" if none). */
const char* wt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WT_H */
