/*
 * cfd.h -- C ABI of libcfd: the per-cell residual, third-order Runge-Kutta
 * update and block-to-block ghost fill of a 3-D multi-block structured-grid
 * compressible flow solver, on one MI355X (gfx950).
 *
 * The operation (Wang et al., "Performance optimizations for scalable CFD
 * applications on hybrid CPU+MIC heterogeneous computing system with millions
 * of cores", Computers & Fluids):
 *   - Section 2.1, Eq. (1): Navier-Stokes equations in curvilinear coordinates,
 *     Q = (rho, rho u, rho v, rho w, rho E);
 *   - Section 2.2, Eq. (3): semi-discrete form dQ/dt = -R(Q);
 *   - Section 2.2, Eqs. (4)-(6): third-order Runge-Kutta with lambda = -dt;
 *   - Sections 2.3 and 3.2.3: multi-block domains whose neighbouring blocks
 *     exchange boundary data after every update.
 * The paper leaves the spatial operator's details open; this library uses a
 * cell-centred finite-volume residual: kappa = 1/3 MUSCL reconstruction of
 * primitive variables with a smooth van Albada-type limiter, Roe's flux with
 * Harten's entropy fix, and face-gradient viscous fluxes (Sutherland's law,
 * constant Prandtl number) on face-area-vector metrics.
 *
 * Conventions
 *   - All device pointers are HIP device memory owned by the caller.  The
 *     library allocates no device memory: everything it needs lives in the
 *     caller's workspace buffer, which must outlive the context.
 *   - All calls are asynchronous on the given stream unless stated.
 *   - Every call returns a cfd_status; no C++ exception crosses the ABI.
 *     After a failure, cfd_last_error() describes it.
 *   - A context is not thread-safe; calls that use one context on one
 *     stream are ordered by that stream.
 *   - Directions 0,1,2 = i,j,k; faces 0..5 = -i,+i,-j,+j,-k,+k.  Patch
 *     ranges on a face are half-open cell ranges in the two transverse
 *     directions in ascending order (i-face: j,k; j-face: i,k; k-face: i,j).
 *   - State layout ("arena"): per block, FP64 structure-of-arrays
 *     [var 0..4][k][j][i] including g ghost layers on every side, i fastest,
 *     rows padded to 16 doubles, interior i = 0 aligned to 128 bytes.
 *     cfd_layout() gives each block's offset and strides.
 */
#ifndef CFD_H
#define CFD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CFD_OK = 0,
  CFD_EINVAL = -1,        /* bad argument, table or size                        */
  CFD_ENOMEM = -2,        /* workspace or output array too small                */
  CFD_EHIP = -3,          /* a HIP runtime call failed                          */
  CFD_ENONFINITE = -4,    /* NaN or Inf found in the state or residual          */
  CFD_ESTATE = -5,        /* call not valid in the context's current state      */
  CFD_EUNSUPPORTED = -6,  /* option not supported                               */
  CFD_EINTERNAL = -7
} cfd_status;

typedef struct cfd_ctx cfd_ctx;

typedef struct { int32_t ni, nj, nk; } cfd_dims;   /* interior cells, each >= ghost_layers */

/* One-to-one block connection, identity orientation.  Fills the ghost cells
 * of `face` of `blk` over the patch [lo, hi) from the cells of `nbr` just
 * inside `nbr_face`, which must be the opposite face of the same direction.
 * Transverse index p maps to p - lo + nbr_lo on the neighbour.  `shift` is
 * added to the neighbour's node coordinates (periodic translation).  Each
 * side of a seam is listed separately.  (Sections 2.3, 3.2.3.) */
typedef struct {
  int32_t blk, face, nbr, nbr_face;
  int32_t lo[2], hi[2], nbr_lo[2];
  double shift[3];
} cfd_conn;

/* Physical boundary patch (the paper specifies none; these are the
 * library's): far field by Riemann invariants, slip wall, no-slip adiabatic
 * wall, zeroth-order extrapolation.  mach > 0 gives a far-field patch its own
 * freestream Mach number (flow angles from cfd_params), so blocks of one
 * context can carry different inflow conditions; mach <= 0 uses
 * cfd_params.mach. */
typedef enum { CFD_BC_FARFIELD = 1, CFD_BC_SLIPWALL = 2, CFD_BC_NOSLIP_ADIABATIC = 3,
               CFD_BC_EXTRAP = 4 } cfd_bc_kind;
typedef struct { int32_t blk, face, kind; int32_t lo[2], hi[2]; int32_t pad; double mach; } cfd_bc;

/* Non-dimensional flow parameters: rho_inf = p_inf = 1, T = p/rho,
 * |u_inf| = mach*sqrt(gamma) along (cos a cos b, sin a cos b, sin b),
 * mu_inf = |u_inf| / reynolds (unit length), Sutherland constant S* = T_s/T_inf.
 * cfl: Courant number of the time step; entropy_fix: Harten delta factor;
 * limiter_eps: limiter regulariser.  viscous: 0 Euler, 1 Navier-Stokes.
 * flux_fp32: 1 evaluates reconstruction and face fluxes in FP32 (state,
 * metrics, flux sums, update and norms stay FP64).  local_dt: 1 uses the
 * per-cell time step (steady problems).  ghost_layers must be 2. */
typedef struct {
  double gamma, prandtl, mach, alpha, beta, reynolds, sutherland, cfl, entropy_fix, limiter_eps;
  int32_t viscous, flux_fp32, local_dt, ghost_layers;
} cfd_params;

/* Tuning knobs of the stage kernels.  Any value changes speed only: the
 * state is bitwise identical across all valid settings, and so are the
 * history's time step, max |R_rho| and conserved totals (sum V Q is reduced
 * over a fixed cut of the grid's 64-cell row chunks that does not depend on
 * the tiles); the L2 norms of R are sums in an order that depends on the
 * kernel and tiles, so across settings they agree to rounding (and bitwise
 * run to run).
 * kernel: 0 = tiled face-once kernel, 1 = simple per-cell kernel,
 *   2 = plane-ring face-once kernel (a ring of three primitive planes in LDS,
 *   two barriers per plane; tile_j = 4 or 8).
 * tile_j, tile_k: tile extent in j and k (tile_i is 64, one wavefront);
 *   the tiled kernel takes tile_j = 2, 4 or 8.  Defaults (set by
 *   cfd_create_blocks): kernel 2, tile_j 8, tile_k 32 (16 for FP32-flux
 *   Euler, whose kernels hold two workgroups per CU), use_graph 1, order 1;
 *   tile_k is halved (down to 4) while the grid gives fewer tiles than CUs,
 *   and a grid with fewer tiles than CUs even then gets the tiled kernel
 *   with tile_j 4 and tile_k halved (down to 1) until it has four tiles per
 *   CU.
 * use_graph: 1 captures one time step in a hipGraph and replays it.
 * order: tile work-list order.  0 = largest tiles first (balances uneven
 *   blocks); 1 = XCD-aware: the tiles are cut into 8 spatially contiguous
 *   chunks and interleaved so that every workgroup of the persistent grid on
 *   one XCD (workgroup id mod 8) works inside one chunk, keeping halo reuse in
 *   that XCD's L2. */
typedef struct { int32_t kernel, tile_j, tile_k, use_graph, order; } cfd_tuning;

/* Arena layout for `nblk` blocks: block_offset[b] = element index of padded
 * cell (i,j,k) = (-g,-g,-g), var 0; block_strides[4*b + 0..3] = element
 * strides of (var, k, j, i).  arena_elems = doubles in one state arena.
 * Output arrays may be NULL.  Host-only, synchronous. */
cfd_status cfd_layout(int32_t nblk, const cfd_dims* dims, int32_t ghost_layers,
                      int64_t* block_offset, int64_t* block_strides, int64_t* arena_elems);

/* Bytes of device workspace cfd_create_blocks needs (metrics; for viscous
 * flow also the viscous face metrics, 21 doubles per padded cell; two stage
 * arenas, tables, reduction partials).  Host-only, synchronous. */
cfd_status cfd_workspace_size(const cfd_params* params, int32_t nblk, const cfd_dims* dims,
                              size_t* workspace_bytes);

/* Build a context: validate the tables (every boundary cell face covered
 * exactly once, ranges in bounds, connected extents match), fill ghost
 * nodes, compute face vectors and volumes (metrics) into the workspace
 * (for viscous flow also the face-averaged transverse face vectors and the
 * auxiliary-cell volumes of the face gradients) and build the tile list.  nodes_dev[b] points to block b's node coordinates,
 * FP64 [3][nk+1][nj+1][ni+1], device memory; they may be freed on return.
 * Synchronises `stream` before returning.  On error *out is NULL. */
cfd_status cfd_create_blocks(const cfd_params* params, int32_t nblk, const cfd_dims* dims,
                             const double* const* nodes_dev, int32_t nconn, const cfd_conn* conns,
                             int32_t nbc, const cfd_bc* bcs, void* workspace_dev,
                             size_t workspace_bytes, hipStream_t stream, cfd_ctx** out);

cfd_status cfd_destroy(cfd_ctx* ctx);

/* Replace the tuning knobs (default {0, 4, 32, 1, 1}).  Drops cached graphs. */
cfd_status cfd_set_tuning(cfd_ctx* ctx, const cfd_tuning* tuning);
cfd_status cfd_get_tuning(const cfd_ctx* ctx, cfd_tuning* tuning);

/* Fill the ghost cells of every block of q_arena_dev (three sweeps i, j, k;
 * connections copy bitwise, physical patches apply their condition).
 * Interior cells are not modified. */
cfd_status cfd_fill_ghosts(cfd_ctx* ctx, double* q_arena_dev, hipStream_t stream);

/* R(Q) = (1/V) sum over the cell's faces of (F_inv - F_vis) . S_out for all
 * interior cells (Eq. 3 with dQ/dt = -R).  Reads the ghost cells of
 * q_arena_dev as they are: call cfd_fill_ghosts first.  r_arena_dev has the
 * state layout; its ghost and padding entries are not written. */
cfd_status cfd_residual(cfd_ctx* ctx, const double* q_arena_dev, double* r_arena_dev,
                        hipStream_t stream);

/* Advance q_arena_dev by nsteps third-order Runge-Kutta steps (Eqs. 4-6,
 * lambda = -dt) with a ghost fill before every stage and the CFL time step
 * recomputed from Q^n at every step.  Ghost cells of q_arena_dev are
 * overwritten.  For inviscid flow the fill covers every face's ghost layers
 * over the face's own cells in one launch: the edge and corner ghost cells,
 * which no inviscid stencil reads, keep their values (cfd_fill_ghosts fills
 * them).  hist_dev (device, nullable) receives one row of 12 doubles
 * per step, all about the state at the start of that step:
 *   [dt, L2(R) x5, sum V Q x5, max|R_rho|],  L2(R_c) = sqrt(sum R_c^2 / N).
 * With local_dt, dt is the minimum of the per-cell steps. */
cfd_status cfd_step(cfd_ctx* ctx, double* q_arena_dev, int32_t nsteps, double* hist_dev,
                    hipStream_t stream);

/* Implicit steps on the finite-volume residual (the sparse linear solve per
 * step that Section 2.3's flowchart names, without its method; this reading
 * is data parallel): backward Euler
 *   (V_c / dt_c + d(V R)_c / dQ) dQ = -V_c R_c
 * with dt_c the CFL step of cfd_step's reading at Courant number `cfl` (per
 * cell with local_dt, else the global minimum), the first-order flux-split
 * approximate Jacobian at every face f between cells L and R (flux
 * (F(Q_L) + F(Q_R)) . S_f / 2 - mu_f (Q_R - Q_L), dissipation frozen at Q^n:
 * mu_f = lambda_f / 2 + lv_f, lambda_f = |u_m . S_f| + c_m |S_f| of the mean
 * primitive state of the two cells, for viscous flow lv_f = max(4/3, gamma/Pr)
 * (mean mu/rho) |S_f|^2 / (mean V)), relaxed by `sweeps` point-Jacobi sweeps
 * from dQ = -V R / D, D_c = V_c / dt_c + the cell's six mu_f; the update is
 * copied across block connections and is zero in the ghost cells of physical
 * boundaries (the boundary conditions act through the residual); then
 * Q += dQ.  nsteps times, in place on q_arena_dev; hist_dev (nullable) gets
 * one row per step as for cfd_step (dt = the least per-cell step).
 * work_dev: cfd_implicit_work_size() bytes of device memory, 256-byte
 * aligned, not overlapping the state (the residual, two update iterates, the
 * face coefficients, diagonal and per-cell steps, each in the state layout).
 * nsteps >= 0, 0 <= sweeps <= 1000, cfl > 0, else CFD_EINVAL; a short
 * workspace gives CFD_ENOMEM.  Asynchronous on stream. */
cfd_status cfd_implicit_work_size(const cfd_ctx* ctx, size_t* bytes);
cfd_status cfd_step_implicit(cfd_ctx* ctx, double* q_arena_dev, int32_t nsteps, int32_t sweeps, double cfl,
                             void* work_dev, size_t work_bytes, double* hist_dev, hipStream_t stream);

/* Multigrid cycles for steady marches.  The paper's convergence test
 * (Section 2.3) asks for a residual drop, and the explicit stages of Eqs.
 * (4)-(6) damp a fine grid's smooth error modes slowly; the paper names no
 * accelerator.  This is the library's: full approximation storage (FAS) on
 * nested grids with the RK3 step as the smoother.  levels[0] is the grid
 * being solved, levels[l + 1] its coarsening (every extent halved: the coarse
 * grid keeps every second node, the connection and boundary tables every
 * range halved; the caller builds it as its own context with cfd_create_blocks
 * and the same parameters).  q_levels[l]: a state arena of level l
 * (q_levels[0] is the state advanced; the others are working states).
 *
 * One V-cycle: going down, on each level l, `pre` RK3 steps of
 * dQ/dt = -(R_l(Q) + F_l) with the level's own CFL steps (F_0 = 0; the
 * coarsest level takes `coarse` steps); then the next level's state
 * Q^0 = sum_children V Q / sum_children V and forcing
 * F_{l+1} = sum_children V (R_l + F_l) / V_{l+1} - R_{l+1}(Q^0) (so that a
 * level whose residual vanishes sees none on the coarse grid); going up,
 * Q_l += Q_{l+1} - Q^0_{l+1} on each coarse cell's 8 children.  With one level
 * a cycle is `coarse` plain RK3 steps.  hist (device, may be NULL):
 * [ncycles][12] rows of cfd_step's layout, each the finest level's first step
 * of the cycle (R without forcing).  Each level runs its own context's
 * tuning (cfd_set_tuning on that context); every tuning gives bitwise the
 * same cycle.
 *
 * cfd_mg_work_size: bytes of work for the hierarchy (three state-layout
 * arenas per level).  cfd_mg_cycles: work_dev 256-byte aligned, disjoint
 * from every level's state; CFD_EINVAL on a hierarchy whose extents do not
 * halve, different block counts or flow parameters, nlevels outside [1, 16],
 * pre or coarse outside [0, 1000], overlapping states; CFD_ENOMEM on a short
 * workspace.  Asynchronous on stream. */
cfd_status cfd_mg_work_size(cfd_ctx* const* levels, int32_t nlevels, size_t* bytes);
cfd_status cfd_mg_cycles(cfd_ctx* const* levels, double* const* q_levels, int32_t nlevels, int32_t pre,
                         int32_t coarse, int32_t ncycles, void* work_dev, size_t work_bytes, double* hist_dev,
                         hipStream_t stream);

/* Norms: out[0..4] = L2 of r (0 if r_arena_dev is NULL), out[5..9] = sum V q,
 * out[10] = max |r_rho|, out[11] = count of non-finite values in q and r.
 * Deterministic fixed-order reductions.  flags & CFD_NORMS_HOST: `out` is
 * host memory and the call synchronises `stream`; then CFD_ENONFINITE is
 * returned if out[11] > 0.  Otherwise `out` is device memory. */
#define CFD_NORMS_HOST 1
cfd_status cfd_norms(cfd_ctx* ctx, const double* q_arena_dev, const double* r_arena_dev,
                     double* out, int32_t flags, hipStream_t stream);

/* Global (minimum) time step of q_arena_dev written to dt_dev (device, one
 * double); with local_dt, the per-cell steps are also kept in the workspace. */
cfd_status cfd_time_step(cfd_ctx* ctx, const double* q_arena_dev, double* dt_dev,
                         hipStream_t stream);

/* Kernel timing.  With profiling on, cfd_step runs without its graph and
 * records a hipEvent pair around every launch of the residual/stage kernel,
 * the ghost-fill sweeps, the time-step kernel and the norms kernel, on the
 * stream they run on.  cfd_profile_read synchronises those events and writes,
 * per kernel class (0 = stage, 1 = ghost-fill sweep, 2 = time step,
 * 3 = norms):
 *   out[4*c + 0] = launches, [4*c + 1] = total ms, [+2] = min ms, [+3] = max ms,
 * then clears the record.  Turning profiling off also clears it. */
cfd_status cfd_set_profiling(cfd_ctx* ctx, int32_t enable);
cfd_status cfd_profile_read(cfd_ctx* ctx, double out[16]);

/* Copy block blk's metrics to out_dev (device) as a dense FP64 array
 * [10][nk+2g][nj+2g][ni+2g]: components 0-2 = S_i, 3-5 = S_j, 6-8 = S_k (the
 * area vectors of the cell's lower i, j, k faces, pointing towards increasing
 * index), 9 = V, ghost cells included.  S_d = 1/2 (x[+t1+t2] - x[0]) x
 * (x[+t2] - x[+t1]) with (t1, t2) cyclic after d; V by the divergence theorem
 * (the geometric conservation requirement of Section 2.2). */
cfd_status cfd_copy_metrics(cfd_ctx* ctx, int32_t blk, double* out_dev, hipStream_t stream);

/* ------------------------------------------------------ split and regroup
 * Load balance by re-partitioning (Section 3.2.1): the blocks of the grid are
 * cut into smaller pieces, and the pieces are dealt into balanced groups, one
 * per device.  The paper leaves the algorithm to a pre-processing tool that it
 * does not print; these are the library's rules.  All three calls are
 * host-only and synchronous and touch no device; output arrays are the
 * caller's.  An output array may be NULL: the call then only stores the
 * count.  An array too small for the count gives CFD_ENOMEM and is left
 * unwritten (the count is stored; call again with a larger array). */
typedef struct { int32_t parent; int32_t lo[3]; int32_t n[3]; } cfd_piece;   /* cells lo .. lo+n-1 of parent */

/* Split plan.  A block of more than max_cells cells is cut in two across its
 * longest index direction (equal extents: the higher direction, k before j
 * before i); both parts are split again by the same rule.  A part whose every
 * extent is below 2*min_width is kept whole, however large.  The lower part
 * takes the multiple of align[d] nearest n/2 (equal distance: the lower) when
 * that lies in [n/4, 3n/4] and leaves both parts min_width cells, else
 * floor(n/2): align = {64, 8, 1} keeps cuts on the stage kernels' tile grid.
 * Pieces are listed block by block, depth first, lower part first.
 * max_cells >= 1; min_width >= 2 (the ghost depth); align may be NULL (all 1),
 * else each entry in [1, 2^20]. */
cfd_status cfd_split_plan(int32_t nblk, const cfd_dims* dims, int64_t max_cells, int32_t min_width,
                          const int32_t align[3], cfd_piece* pieces, int32_t capacity, int32_t* npieces);

/* Connection and boundary tables of a set of pieces that tiles every block
 * (checked: every cell exactly once).  A piece face inside its parent becomes
 * a connection to each sibling piece across it (zero shift, both sides
 * listed); a piece face on its parent's face takes the parent's boundary
 * patches and connections there, cut to the piece, and each connection is
 * cut again to every piece of the neighbour block that it reaches (shift
 * kept).  The parent tables are checked as cfd_create_blocks checks them.
 * With the pieces' nodes and states sliced from their parents, the solver
 * gives the pieces bitwise the same state as the parent blocks. */
cfd_status cfd_split_tables(int32_t nblk, const cfd_dims* dims, const cfd_conn* conns, int32_t nconn,
                            const cfd_bc* bcs, int32_t nbc, const cfd_piece* pieces, int32_t npieces,
                            cfd_conn* out_conns, int32_t conn_capacity, int32_t* nconn_out, cfd_bc* out_bcs,
                            int32_t bc_capacity, int32_t* nbc_out);

/* Regroup by longest processing time first (Graham, 1969): items in
 * decreasing load (equal loads: lower index first) each go to the group g
 * whose (load after taking the item) / capacity[g] is least (equal: lower g;
 * computed in FP64).  capacity (may be NULL: all 1) carries the paper's load
 * ratio between unlike devices; with equal capacities the largest group load
 * is at most (4/3 - 1/(3 ngroups)) times the optimum.  group[i] in
 * [0, ngroups); group_load (may be NULL) receives each group's total. */
cfd_status cfd_regroup(int32_t n, const int64_t* load, int32_t ngroups, const double* capacity,
                       int32_t* group, int64_t* group_load);

/* ---------------------------------------------------------- high order
 * Sixth-order staggered flux difference, Section 2.2, Eq. (2): the
 * cell-centred derivative along index direction d (0, 1, 2 = i, j, k) of a
 * face-centred field, for the n[0] x n[1] x n[2] cells of one block,
 *   out_i = [75/64 (F_{i+1/2} - F_{i-1/2}) - 25/384 (F_{i+3/2} - F_{i-3/2})
 *            + 3/640 (F_{i+5/2} - F_{i-5/2})] / h.
 * f_dev: nvar dense arrays [k][j][i] (i fastest) with n[d] + 5 entries along
 *   d (the faces i - 1/2 for i = -2 .. n[d] + 2) and n[t] along the other
 *   directions t.  The two faces beyond the block on each side are the
 *   caller's to supply: the paper's block closures are in references it does
 *   not reproduce, so the residual kernels above do not use this operator.
 * out_dev: nvar dense arrays [k][j][i] of n[0] x n[1] x n[2] cells.
 * Both are the caller's device memory and must not overlap.  n[t] >= 1,
 * 1 <= nvar <= 64, h > 0 and finite, else CFD_EINVAL.  Asynchronous on
 * stream. */
cfd_status cfd_staggered_diff6(const double* f_dev, double* out_dev, const int32_t n[3], int32_t d, int32_t nvar,
                               double h, hipStream_t stream);

/* Fifth-order weighted cell-edge interpolation of WCNS-E-5, the scheme
 * Section 2.2 names for the face states (its reference gives the
 * construction; this is that published construction, not a formula the paper
 * prints): left and right states at the n[d] + 5 faces i - 1/2,
 * i = -2 .. n[d] + 2, of the n[0] x n[1] x n[2] cells of one block, the input
 * of cfd_staggered_diff6 after a flux function.  The left state at the face
 * between cells c and c + 1 combines three 3-cell candidates
 * u_c + g/2 + s/8 (one-sided and central first and second differences g, s of
 * the stencils ending, centred and starting at c) with weights
 * d_k / (eps + g_k^2 + s_k^2)^2, d = (1/16, 10/16, 5/16), normalised; the
 * right state is the mirror image about the face.  With smooth data the
 * weights tend to d: the 5-cell interpolation, fifth order.
 * u_dev: nvar dense arrays [k][j][i] with n[d] + 10 cells along d (cells
 *   -5 .. n[d] + 4: five beyond the block on each side, the caller's) and
 *   n[t] along the other directions.
 * left_dev, right_dev: nvar dense arrays with n[d] + 5 faces along d.
 * All the caller's device memory, pairwise disjoint.  n[t] >= 1,
 * 1 <= nvar <= 64, eps > 0 and finite (1e-6 is usual), else CFD_EINVAL.
 * Asynchronous on stream. */
cfd_status cfd_wcns5_edges(const double* u_dev, double* left_dev, double* right_dev, const int32_t n[3], int32_t d,
                           int32_t nvar, double eps, hipStream_t stream);

/* Inviscid WCNS-E-5 residual of one block periodic in all three directions on
 * a uniform Cartesian grid (spacings h[0..2] along i, j, k): for each
 * direction, the primitive variables padded periodically, their WCNS-E-5 face
 * states (cfd_wcns5_edges), Roe's flux per unit area through each face (the
 * flux splitting of the residual kernels, Harten factor entropy_fix), and
 * Eq. (2) (cfd_staggered_diff6); R = the sum over directions, so that
 * dQ/dt = -R (Section 2.2, Eq. 3 with the paper's spatial operator).  The
 * face states and Roe's flux are formed in one pass, the states staying in
 * registers.  Curvilinear blocks: cfd_wcns5_euler_residual_curv_periodic below.
 * q_dev, r_dev: [5][nk][nj][ni] dense FP64 (conserved variables, residual);
 * work_dev: cfd_wcns5_euler_work_bytes() bytes of device memory (the padded
 * primitives and the face flux of the largest direction).  All the
 * caller's, pairwise disjoint.  n[t] >= 1, h > 0, gamma > 1, entropy_fix >= 0,
 * eps > 0, else CFD_EINVAL; a short workspace gives CFD_ENOMEM.
 * Asynchronous on stream. */
cfd_status cfd_wcns5_euler_work_bytes(const int32_t n[3], size_t* bytes);
cfd_status cfd_wcns5_euler_residual_periodic(const double* q_dev, double* r_dev, void* work_dev, size_t work_bytes,
                                            const int32_t n[3], const double h[3], double gamma, double entropy_fix,
                                            double eps, hipStream_t stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the residual of
 * cfd_wcns5_euler_residual_periodic, bitwise the same, with its scratch (the
 * padded primitives and one direction's face flux) in a static device array
 * of CFD_WCNS5_NOALLOC_MAX_BYTES bytes that the library holds on every device
 * it runs on until the process ends.  No workspace argument: the call
 * allocates nothing and calls no allocating routine.  A block whose
 * cfd_wcns5_euler_work_bytes() exceeds the maximum (about 90^3 cells) gives
 * CFD_ENOMEM before any launch.  q_dev, r_dev and the stream must be on the
 * device current on the calling thread (else CFD_EINVAL).  The array is
 * overwritten in full by every call (nothing in it has to start at zero), and
 * all calls on one device share it: calls that overlap in time on one device
 * (different streams, or threads) race and give undefined results; order
 * them on one stream.  Other arguments and errors as for
 * cfd_wcns5_euler_residual_periodic.  Asynchronous on stream. */
#define CFD_WCNS5_NOALLOC_MAX_BYTES ((size_t)64 << 20)
cfd_status cfd_wcns5_euler_residual_periodic_noalloc(const double* q_dev, double* r_dev, const int32_t n[3],
                                                     const double h[3], double gamma, double entropy_fix,
                                                     double eps, hipStream_t stream);

/* Metrics of one curvilinear block periodic in all three directions, for the
 * geometric conservation law that Section 2.2 requires of the scheme on
 * curvilinear grids (the paper defers the formulas to its reference; this is
 * the symmetric conservative form).  Vertex v along a direction sits at index
 * position v + 1/2, cell centres at integer positions; D is Eq. (2) with
 * h = 1 and I the sixth-order mid-point interpolation
 * (150 (f_{+1/2} + f_{-1/2}) - 25 (f_{+3/2} + f_{-3/2}) + 3 (f_{+5/2} + f_{-5/2})) / 256.
 * The area vector of face v + 1/2 of direction d is
 *   S_d = 1/2 [D_b (D_a X x I_a X) - D_a (D_b X x I_b X)],  (a, b) = (d+1, d+2) mod 3,
 * so sum_d D_d S_d = 0 at every cell to rounding (a uniform stream stays
 * uniform); J^{-1} = det[X_xi, X_eta, X_zeta] at the cell centre, each column
 * D along its direction of the coordinates interpolated (I) along the other
 * two.  Both are exact for maps of total degree 3.
 * xv_dev: [3][nk][nj][ni] vertex coordinates (x, y, z); vertex (i, j, k) is
 *   the upper corner of cell (i, j, k).  period: host, 9 doubles, period[3d + c]
 *   = component c of the grid's displacement over one period along direction
 *   d (vertex v + n_d along d = vertex v + that displacement).
 * s_dev: [3 (d)][3 (x, y, z)][nk][nj][ni] out: S_d of face v + 1/2 at index v
 *   along d.  jinv_dev: [nk][nj][ni] out.
 * All the caller's device memory, pairwise disjoint.  n[t] >= 1, at most 2^34
 * cells, finite periods, else CFD_EINVAL.  Asynchronous on stream. */
cfd_status cfd_wcns5_metrics_periodic(const double* xv_dev, const double period[9], const int32_t n[3], double* s_dev,
                                      double* jinv_dev, hipStream_t stream);

/* The inviscid WCNS-E-5 residual of a periodic curvilinear block: as
 * cfd_wcns5_euler_residual_periodic, with Roe's flux through each face's
 * area vector S_d (flux times |S_d|), Eq. (2) in index units, and the sum over
 * directions divided by J^{-1}: R = J sum_d D_d F_d, dQ/dt = -R.  On a uniform
 * Cartesian grid it reduces to the Cartesian residual.  s_dev, jinv_dev from
 * cfd_wcns5_metrics_periodic (J^{-1} must not vanish); the workspace is
 * cfd_wcns5_euler_work_bytes() bytes; the other arguments and errors as for
 * the Cartesian residual, and r and the workspace must not overlap the
 * metrics.  Asynchronous on stream. */
cfd_status cfd_wcns5_euler_residual_curv_periodic(const double* q_dev, const double* s_dev, const double* jinv_dev,
                                                  double* r_dev, void* work_dev, size_t work_bytes,
                                                  const int32_t n[3], double gamma, double entropy_fix, double eps,
                                                  hipStream_t stream);

/* nsteps third-order Runge-Kutta steps (Section 2.2, Eqs. 4-6, lambda = -dt,
 * fixed dt) of dQ/dt = -R(Q) with the periodic WCNS-E-5 residual above, in
 * place on q_dev ([5][nk][nj][ni]).  work_dev: cfd_wcns5_euler_step_work_bytes()
 * bytes (the residual's workspace, the step's start state and R).  dt > 0,
 * nsteps >= 0, the other arguments as for the residual; a short workspace
 * gives CFD_ENOMEM.  Asynchronous on stream. */
cfd_status cfd_wcns5_euler_step_work_bytes(const int32_t n[3], size_t* bytes);

/* nsteps RK3 steps as cfd_wcns5_euler_steps_periodic, with the curvilinear
 * residual cfd_wcns5_euler_residual_curv_periodic (s_dev, jinv_dev from
 * cfd_wcns5_metrics_periodic; q must not overlap them or the workspace).
 * work_dev: cfd_wcns5_euler_step_work_bytes() bytes.  Errors as for the
 * Cartesian steps and the curvilinear residual.  Asynchronous on stream. */
cfd_status cfd_wcns5_euler_steps_curv_periodic(double* q_dev, const double* s_dev, const double* jinv_dev,
                                               void* work_dev, size_t work_bytes, const int32_t n[3], double gamma,
                                               double entropy_fix, double eps, double dt, int32_t nsteps,
                                               hipStream_t stream);

/* Viscous terms by fourth-order central differencing, which Section 2.2
 * chooses for the viscous flux derivatives (the paper prints no formulas;
 * these are the textbook fourth-order forms on a uniform grid, exact for
 * cubics): on one block periodic in all three directions, adds -div F_v to
 * r_dev (so that after cfd_wcns5_euler_residual_periodic, r is the
 * Navier-Stokes residual, dQ/dt = -R).  (u, v, w, T) and their cell
 * gradients by the central derivative (f_{-2} - 8 f_{-1} + 8 f_1 - f_2) / 12h;
 * at each face the values by (-f_{-1} + 9 f_0 + 9 f_1 - f_2) / 16 (transverse
 * gradients likewise), the normal derivative by
 * (f_{-1} - 27 f_0 + 27 f_1 - f_2) / 24h; the stress with Stokes' hypothesis,
 * Sutherland's viscosity mu_inf T^1.5 (1 + s_star) / (T + s_star), conduction
 * mu gamma / ((gamma - 1) prandtl); -div by the staggered difference
 * (F_{-3/2} - 27 F_{-1/2} + 27 F_{1/2} - F_{3/2}) / 24h.
 * q_dev, r_dev: [5][nk][nj][ni] dense FP64; work_dev:
 * cfd_c4_viscous_work_bytes() bytes.  All the caller's, pairwise disjoint.
 * Asynchronous on stream. */
cfd_status cfd_c4_viscous_work_bytes(const int32_t n[3], size_t* bytes);
cfd_status cfd_c4_viscous_add_periodic(const double* q_dev, double* r_dev, void* work_dev, size_t work_bytes,
                                       const int32_t n[3], const double h[3], double gamma, double prandtl,
                                       double mu_inf, double s_star, hipStream_t stream);
cfd_status cfd_wcns5_euler_steps_periodic(double* q_dev, void* work_dev, size_t work_bytes, const int32_t n[3],
                                          const double h[3], double gamma, double entropy_fix, double eps, double dt,
                                          int32_t nsteps, hipStream_t stream);

/* The fourth-order central viscous terms on a periodic curvilinear block
 * (Section 2.2's choice for the viscous flux derivatives, on the metrics of
 * cfd_wcns5_metrics_periodic): index derivatives of u, v, w, T at the cells;
 * the metrics S_t at the cells from their faces along t,
 * (-S_{i-3/2} + 9 S_{i-1/2} + 9 S_{i+1/2} - S_{i+3/2}) / 16; at each face of
 * direction d the physical gradient J sum_t S_t d/dxi_t (compact derivative
 * along d, face values of the cell derivatives, of S_t (t != d) and of J^{-1});
 * stress, Sutherland viscosity and conduction as above, the viscous flux
 * through S_d; r -= J times the staggered difference, summed over d.  On a
 * uniform Cartesian grid this equals cfd_c4_viscous_add_periodic.
 * q_dev, r_dev: [5][nk][nj][ni]; s_dev, jinv_dev from the metrics call;
 * work_dev: cfd_c4_viscous_curv_work_bytes() bytes (37 doubles per cell: u,
 * v, w, T and their index derivatives, then the face metrics of the three
 * directions, formed from s and J^{-1} on each call).  r and the workspace
 * must not overlap each other, q or the metrics.  Errors as for the Cartesian
 * terms.  Asynchronous on stream. */
cfd_status cfd_c4_viscous_curv_work_bytes(const int32_t n[3], size_t* bytes);
cfd_status cfd_c4_viscous_add_curv_periodic(const double* q_dev, const double* s_dev, const double* jinv_dev,
                                            double* r_dev, void* work_dev, size_t work_bytes, const int32_t n[3],
                                            double gamma, double prandtl, double mu_inf, double s_star,
                                            hipStream_t stream);

/* Curvilinear blocks joined face to face (Section 2.2 asks for care with the
 * points that adjacent blocks share; this covers whole faces joined with the
 * same index orientation, not physical boundaries).  The scheme's stencils
 * run across every seam unchanged: along each direction the five cells beyond
 * a block come from the neighbour across that face, as do the area vectors of
 * the three faces below and the two above the block.  A periodic block is its
 * own neighbour.
 *
 * cfd_wcns5_metrics_ext: the metrics of cfd_wcns5_metrics_periodic from an
 * explicit array of the block's vertices -3 .. n + 1 along each direction,
 * xe_dev [3][nk + 5][nj + 5][ni + 5] (vertex v at index v + 3), taken by the
 * caller from the whole grid, so the two sides of a seam compute its metrics
 * from the same coordinates.  Outputs and errors as for the periodic call.
 *
 * cfd_wcns5_euler_residual_blocks: the curvilinear residual of nblk blocks.
 * dims: host [nblk][3] (ni, nj, nk); nbr: host [nblk][6], nbr[6b + 2d + side]
 * = the block across face (d, side) of block b (side 0: the low face); the
 * link must be mutual (face f of b <-> face f ^ 1 of the neighbour), the
 * joined faces of equal extents, and every neighbour at least 5 cells across
 * the seam, else CFD_EINVAL.  q_dev, s_dev, jinv_dev, r_dev: host arrays of
 * nblk device pointers ([5][nk][nj][ni], the metrics of each block, its
 * residual out); work_dev: cfd_wcns5_euler_blocks_work_bytes() bytes.  No
 * residual may overlap an input, another residual or the workspace.  gamma,
 * entropy_fix, eps as for the periodic residual.  Asynchronous on stream. */
cfd_status cfd_wcns5_metrics_ext(const double* xe_dev, const int32_t n[3], double* s_dev, double* jinv_dev,
                                 hipStream_t stream);
cfd_status cfd_wcns5_euler_blocks_work_bytes(int32_t nblk, const int32_t* dims, const int32_t* nbr, size_t* bytes);
cfd_status cfd_wcns5_euler_residual_blocks(int32_t nblk, const int32_t* dims, const int32_t* nbr,
                                           const double* const* q_dev, const double* const* s_dev,
                                           const double* const* jinv_dev, double* const* r_dev, void* work_dev,
                                           size_t work_bytes, double gamma, double entropy_fix, double eps,
                                           hipStream_t stream);

/* nsteps RK3 steps (Eqs. 4-6, lambda = -dt, fixed dt) of the Navier-Stokes
 * equations on a periodic curvilinear block, in place on q_dev: each stage's
 * residual is cfd_wcns5_euler_residual_curv_periodic plus the viscous terms
 * of cfd_c4_viscous_add_curv_periodic.  work_dev: cfd_wcns5_ns_step_work_bytes()
 * bytes (the larger of the two scratch areas, which the stage reuses, the
 * viscous face metrics, formed once per call, then the step's start state and
 * R).  Arguments and errors as for those calls and
 * cfd_wcns5_euler_steps_curv_periodic.  Asynchronous on stream. */
cfd_status cfd_wcns5_ns_step_work_bytes(const int32_t n[3], size_t* bytes);
cfd_status cfd_wcns5_ns_steps_curv_periodic(double* q_dev, const double* s_dev, const double* jinv_dev,
                                            void* work_dev, size_t work_bytes, const int32_t n[3], double gamma,
                                            double entropy_fix, double eps, double prandtl, double mu_inf,
                                            double s_star, double dt, int32_t nsteps, hipStream_t stream);

/* Implicit steps on a periodic curvilinear block (the sparse linear solve per
 * step that the paper's flowchart names, without its method; this reading is
 * data parallel): backward Euler (I/dt + dR/dQ) dQ = -R for the residual of
 * cfd_wcns5_euler_residual_curv_periodic, with the flux-split approximate
 * Jacobian A+- = (A +- lambda I)/2 at each face (lambda = |u . S| + c |S| of
 * the mean primitive state of the two cells), relaxed by `sweeps` point-Jacobi
 * sweeps from dQ = -R / D, D = 1/dt + J sum_d (lambda_+ + lambda_-)/2; the
 * off-diagonal products are flux differences F(Q + dQ) . S - F(Q) . S.  With
 * viscous != 0 the residual adds cfd_c4_viscous_add_curv_periodic's terms and
 * the operator a central diffusion split: per face the viscous spectral radius
 * lv = max(4/3, gamma/Pr)(mu/rho)|S|^2 / J^{-1} (means of the two cells) adds
 * J sum_d (lv_+ + lv_-) to D and -(lv_+ dQ_{i+1} + lv_- dQ_{i-1}) to the
 * off-diagonal sum.  Then q += dQ; nsteps times, in place.  work_dev:
 * cfd_wcns5_implicit_step_work_bytes() bytes.  dt > 0, nsteps >= 0,
 * 0 <= sweeps <= 1000, gamma > 1, for viscous flow Pr > 0, mu_inf >= 0,
 * s_star > 0, and q, the metrics and the workspace pairwise disjoint, else
 * CFD_EINVAL; a short workspace gives CFD_ENOMEM.  Asynchronous on stream. */
cfd_status cfd_wcns5_implicit_step_work_bytes(const int32_t n[3], size_t* bytes);
cfd_status cfd_wcns5_implicit_steps_curv_periodic(double* q_dev, const double* s_dev, const double* jinv_dev,
                                                  void* work_dev, size_t work_bytes, const int32_t n[3], double gamma,
                                                  double entropy_fix, double eps, int32_t viscous, double prandtl,
                                                  double mu_inf, double s_star, double dt, int32_t nsteps,
                                                  int32_t sweeps, hipStream_t stream);

/* Implicit steps (those of cfd_wcns5_implicit_steps_curv_periodic, viscous
 * optional) on blocks joined face to face (table, extents and pointer arrays
 * as for cfd_wcns5_euler_residual_blocks; q_dev[b] updated in place): the
 * residual of cfd_wcns5_euler_residual_blocks (plus cfd_c4_viscous_add_blocks
 * when viscous), and every sweep reads the neighbours' states, updates, radii
 * and face metrics across the seams.  Each sweep reads
 * only the previous iterate, so the steps do not depend on how the domain is
 * cut (a split block gives the unsplit block's bits).  work_dev:
 * cfd_wcns5_implicit_blocks_work_bytes() bytes.  Errors as for the periodic
 * call and the table checks; no state may overlap another, the metrics or
 * the workspace.  Asynchronous on stream. */
cfd_status cfd_wcns5_implicit_blocks_work_bytes(int32_t nblk, const int32_t* dims, const int32_t* nbr, size_t* bytes);
cfd_status cfd_wcns5_implicit_steps_blocks(int32_t nblk, const int32_t* dims, const int32_t* nbr, double* const* q_dev,
                                           const double* const* s_dev, const double* const* jinv_dev, void* work_dev,
                                           size_t work_bytes, double gamma, double entropy_fix, double eps,
                                           int32_t viscous, double prandtl, double mu_inf, double s_star, double dt,
                                           int32_t nsteps, int32_t sweeps, hipStream_t stream);

/* RK3 Navier-Stokes steps (Eqs. 4-6, lambda = -dt, fixed dt) on blocks joined
 * face to face, in place on every q_dev[b]: each stage's residual is
 * cfd_wcns5_euler_residual_blocks plus cfd_c4_viscous_add_blocks over all
 * blocks at that stage (table, extents and pointer arrays as for those
 * calls).  work_dev: cfd_wcns5_ns_blocks_work_bytes() bytes (the larger of the
 * residual's and the viscous terms' scratch, then each block's start state
 * and R, then the viscous face metrics, formed once per call).  Errors as for
 * those calls and cfd_wcns5_ns_steps_curv_periodic; no
 * state may overlap another, the metrics or the workspace.  Asynchronous on
 * stream. */
cfd_status cfd_wcns5_ns_blocks_work_bytes(int32_t nblk, const int32_t* dims, const int32_t* nbr, size_t* bytes);
cfd_status cfd_wcns5_ns_steps_blocks(int32_t nblk, const int32_t* dims, const int32_t* nbr, double* const* q_dev,
                                     const double* const* s_dev, const double* const* jinv_dev, void* work_dev,
                                     size_t work_bytes, double gamma, double entropy_fix, double eps, double prandtl,
                                     double mu_inf, double s_star, double dt, int32_t nsteps, hipStream_t stream);

/* Closures of the WCNS-E-5 scheme at walls and the far field (Section 2.2
 * leaves the conditions at block boundaries to its references; this is the
 * library's reading).  An owner block whose faces across one direction
 * `bounded` are physical, and whose other directions are periodic, gets two
 * ghost blocks, CFD_WCNS5_GHOST cells across `bounded` with the owner's
 * transverse extents, joined to its low and high faces in an ordinary
 * joined-block table (the two ghost blocks' far faces joined to each other,
 * so that every link is mutual).  Every stencil of the owner then runs
 * unchanged up to the boundary:
 *
 * cfd_wcns5_extend_vertices: the vertices the owner and its ghost blocks take
 * their metrics from.  xv_dev [3][nk'][nj'][ni']: along a periodic direction
 * d the n_d upper corners 0 .. n_d - 1 (n'_d = n_d; period[3 d + c] is the
 * grid's displacement over one period), along `bounded` the n_d + 1 vertex
 * planes -1 .. n_d - 1 (the boundary surfaces are the first and the last).
 * xe_dev [3][Ek][Ej][Ei]: along a periodic direction E_d = n_d + 5 (vertices
 * -3 .. n_d + 1, vertex v = vertex v mod n_d plus floor(v / n_d) periods);
 * along `bounded` E_d = n_d + 1 + 2 CFD_WCNS5_XLAYERS (planes -1 - XLAYERS ..
 * n_d - 1 + XLAYERS, those beyond the boundary continued linearly from the
 * two planes at that end: x_(b - m) = x_b + m (x_b - x_(b + 1))).  bounded =
 * -1 makes every direction periodic.  The owner's metrics
 * (cfd_wcns5_metrics_ext) come from the window of vertices -3 .. n + 1 along
 * every direction, the low ghost block's from -8 .. 1 along `bounded`, the
 * high one's from n - 3 .. n + 6.  CFD_EINVAL on bad extents, a non-finite
 * period or overlapping input and output.
 *
 * cfd_wcns5_fill_ghost_blocks: the ghost blocks' states from the owner's
 * q_dev [5][nk][nj][ni] (layouts of cfd_wcns5_euler_residual_blocks).  The
 * ghost cell m = 1 .. 5 cells beyond a wall takes the owner cell m - 1
 * inside it with the momentum reflected about the boundary face's unit normal
 * (CFD_BC_SLIPWALL) or negated (CFD_BC_NOSLIP_ADIABATIC), density and energy
 * copied; every layer beyond the far field (CFD_BC_FARFIELD) takes the
 * characteristic state of the owner's first cell (Riemann invariants along the
 * outward normal, freestream rho = p = 1 and velocity uinf).  The normal comes
 * from the face metrics: the low ghost block's last face (s_lo_dev) and the
 * owner's last face (s_dev).  kind[0]: the low face, kind[1]: the high face.
 * CFD_EINVAL on a bad argument or when a ghost state overlaps the owner's
 * state, a metric array or the other ghost state.
 *
 * Owners that tile the periodic directions (as blocks of the one-GPU share
 * tile x and z) each get their own two ghost blocks; a ghost block joins the
 * same-side ghost block of its owner's neighbour across the cut, so the
 * tiling's ghost layers are those of the untiled block cut the same way.
 *
 * cfd_wcns5_steps_blocks_closed: cfd_wcns5_ns_steps_blocks with the ghost
 * blocks of the nclosures closures[] refilled before every stage's residual
 * and the viscous terms only when viscous != 0 (same workspace size).  Each
 * closure is checked against the table (distinct blocks in range, ghost
 * extents, the ghost blocks joined to the owner's two faces across
 * `bounded`).  Closures are applied in list order; a block may be the ghost
 * block of one closure only, and the owner of a closure may be the ghost
 * block of an earlier one (corners), not of a later one.  The ghost blocks'
 * own states after a call are scratch: being refilled before every stage,
 * they skip their own faces, differences and updates.  Asynchronous on
 * stream. */
#define CFD_WCNS5_GHOST 5
#define CFD_WCNS5_XLAYERS 7
typedef struct {
  int32_t owner, ghost_lo, ghost_hi;   /* block indices in the joined-block table */
  int32_t bounded;                     /* the direction 0..2 whose two faces are physical */
  int32_t kind[2];                     /* cfd_bc_kind of the low and the high face */
  double uinf[3];                      /* far-field velocity (rho = p = 1) */
} cfd_wcns5_closure;
cfd_status cfd_wcns5_extend_vertices(const double* xv_dev, const int32_t n[3], int32_t bounded,
                                     const double period[9], double* xe_dev, hipStream_t stream);
/* The same for one or two bounded directions, bit d of bounded_mask set for a
 * bounded direction d (at most two bits; 0: all periodic).  With two, the
 * lower direction is continued first and the second from those values, so
 * the vertices past two ends (the corner ghost blocks') continue the
 * continued planes.  A block closed across two directions has, besides its
 * four face ghost blocks, four corner ghost blocks CFD_WCNS5_GHOST cells
 * across both; a corner is filled by a closure whose owner is the face ghost
 * block across the lower direction (its cells mirrored across the higher
 * direction's boundary), listed after the closure that fills that face ghost
 * block: the sweep order of the finite-volume ghost fill. */
cfd_status cfd_wcns5_extend_vertices_mask(const double* xv_dev, const int32_t n[3], int32_t bounded_mask,
                                          const double period[9], double* xe_dev, hipStream_t stream);
cfd_status cfd_wcns5_fill_ghost_blocks(const double* q_dev, double* q_lo_dev, double* q_hi_dev, const double* s_dev,
                                       const double* s_lo_dev, const int32_t n[3], int32_t bounded,
                                       const int32_t kind[2], double gamma, const double uinf[3],
                                       hipStream_t stream);
cfd_status cfd_wcns5_steps_blocks_closed(int32_t nblk, const int32_t* dims, const int32_t* nbr, double* const* q_dev,
                                         const double* const* s_dev, const double* const* jinv_dev,
                                         const cfd_wcns5_closure* closures, int32_t nclosures, int32_t viscous,
                                         void* work_dev, size_t work_bytes, double gamma, double entropy_fix, double eps,
                                         double prandtl, double mu_inf, double s_star, double dt, int32_t nsteps,
                                         hipStream_t stream);

/* The fourth-order viscous terms of cfd_c4_viscous_add_curv_periodic on blocks
 * joined face to face (the table, extents and pointer arrays as for
 * cfd_wcns5_euler_residual_blocks): every four-point stencil runs across the
 * seams, reading the neighbours' u, v, w, T, cell derivatives, cell metrics,
 * J^{-1} and face metrics; adds -div F_v to each r_dev[b].  work_dev:
 * cfd_c4_viscous_blocks_work_bytes() bytes (37 doubles per cell of every
 * block, as for the periodic call).  Gas parameters and errors as for the
 * periodic call.  Asynchronous on stream. */
cfd_status cfd_c4_viscous_blocks_work_bytes(int32_t nblk, const int32_t* dims, const int32_t* nbr, size_t* bytes);
cfd_status cfd_c4_viscous_add_blocks(int32_t nblk, const int32_t* dims, const int32_t* nbr, const double* const* q_dev,
                                     const double* const* s_dev, const double* const* jinv_dev, double* const* r_dev,
                                     void* work_dev, size_t work_bytes, double gamma, double prandtl, double mu_inf,
                                     double s_star, hipStream_t stream);

/* The global time step of a periodic curvilinear block for the RK3 steps
 * above (the paper leaves the step size of Eqs. 4-6 open; the finite-volume
 * path's reading): per cell dt_c = cfl J^{-1} / (sum_d L_d + 4 sum_d Lv_d),
 * L_d = |u . Sb_d| + c |Sb_d|, Lv_d = max(4/3, gamma/Pr)(mu/rho)|Sb_d|^2 / J^{-1}
 * when viscous != 0 (Sutherland's mu from mu_inf, s_star), Sb_d the mean of the
 * cell's two d-face area vectors; *dt_dev = the least dt_c (0 if a cell is
 * non-physical or has J^{-1} <= 0).  q_dev [5][nk][nj][ni]; s_dev, jinv_dev
 * from cfd_wcns5_metrics_periodic; dt_dev: one 8-byte aligned device double,
 * the caller's, not overlapping the inputs.  gamma > 1, cfl > 0, and for
 * viscous flow Pr > 0, mu_inf >= 0, s_star > 0, else CFD_EINVAL.
 * Asynchronous on stream: read *dt_dev after the stream has run it. */
cfd_status cfd_wcns5_time_step_curv_periodic(const double* q_dev, const double* s_dev, const double* jinv_dev,
                                             const int32_t n[3], double gamma, double cfl, int32_t viscous,
                                             double prandtl, double mu_inf, double s_star, double* dt_dev,
                                             hipStream_t stream);

/* ---------------------------------------------------------------- warm start
 * A multilayer perceptron predicts the steady flow of a channel-bump case
 * from its condition and a cell position, giving the time march a warm start
 * instead of the uniform stream.  (The paper's solver starts from an
 * initialised flow field, Section 2.3, and iterates to convergence; the
 * learned initial field is this library's addition.)
 *   features (5): [(M - 0.675)/0.175, (h - 0.06)/0.04, 2 xi - 1, 2 eta - 1,
 *                  2 zeta - 1], xi = (i + 1/2)/ni etc. over a block's cells;
 *   network: n_hidden SiLU layers of width d_hidden, linear output;
 *   outputs (5): (rho - 1, u - M sqrt(gamma), v, w, p - 1).
 * Inference runs on BF16 matrix cores (MFMA) with FP32 accumulation; training
 * uses FP32 backward kernels with fixed-order reductions and Adam on FP32
 * master weights.  Parameter layout (padded): for each layer W [N][K]
 * (output-major) then b [N]; K of the input layer is 16 (inputs zero
 * padded), N of the output layer is 16 (outputs zero padded).  BF16 values
 * are raw uint16 bit patterns.  Cells are ordered block, k, j, i (i fastest). */
typedef struct { int32_t d_in, d_hidden, n_hidden, d_out, activation; } cfd_mlp_desc;  /* activation 1 = SiLU */

/* Parameter count (padded layout), cache floats per point for training, and
 * the workspace bytes cfd_mlp_mse / cfd_mlp_backward need for n points. */
cfd_status cfd_mlp_sizes(const cfd_mlp_desc* desc, int64_t n, int64_t* n_params, int64_t* cache_per_point,
                         size_t* work_bytes);
/* y[n][d_out] = MLP(x[idx[p]] or x[p]); with cache != NULL also stores each
 * layer's input and pre-activation for cfd_mlp_backward. */
cfd_status cfd_mlp_forward(const cfd_mlp_desc* desc, const uint16_t* params_bf16, const float* x,
                           const int32_t* idx, int64_t n, float* y, float* cache, hipStream_t stream);
/* Mean squared error against t[idx[p]] (or t[p]); dy = d loss / d y;
 * loss_dev (device, 1 double). */
cfd_status cfd_mlp_mse(const cfd_mlp_desc* desc, const float* y, const float* t, const int32_t* idx, int64_t n,
                       float* dy, double* loss_dev, void* work, size_t work_bytes, hipStream_t stream);
/* Gradient of the loss w.r.t. all parameters (padded layout, FP32). */
cfd_status cfd_mlp_backward(const cfd_mlp_desc* desc, const uint16_t* params_bf16, const float* cache,
                            const float* dy, int64_t n, float* grad, void* work, size_t work_bytes,
                            hipStream_t stream);
/* Adam step t (1-based) on the FP32 master weights; refreshes the BF16 copy. */
cfd_status cfd_mlp_adam(const cfd_mlp_desc* desc, float* master, float* m, float* v, const float* grad,
                        uint16_t* params_bf16, float lr, float beta1, float beta2, float eps, int32_t t,
                        hipStream_t stream);
/* BF16 copy of FP32 master weights (round to nearest even). */
cfd_status cfd_mlp_to_bf16(const cfd_mlp_desc* desc, const float* master, uint16_t* params_bf16,
                           hipStream_t stream);
/* Features of every interior cell of every block: x[ncells][5]; cond_dev is
 * [nblk][2] = (inflow Mach, bump height) per block, FP64 device memory. */
cfd_status cfd_mlp_features(cfd_ctx* ctx, const double* cond_dev, float* x, hipStream_t stream);
/* Training targets from a state arena: t[ncells][5] primitive deviations. */
cfd_status cfd_mlp_targets(cfd_ctx* ctx, const double* q_arena_dev, const double* cond_dev, float* t,
                           hipStream_t stream);
/* Write the interior state from network outputs y[ncells][5] (warm start). */
cfd_status cfd_mlp_to_state(cfd_ctx* ctx, const float* y, const double* cond_dev, double* q_arena_dev,
                            hipStream_t stream);

const char* cfd_status_string(cfd_status s);
const char* cfd_last_error(const cfd_ctx* ctx);   /* ctx may be NULL: last global error */

#ifdef __cplusplus
}
#endif
#endif /* CFD_H */
