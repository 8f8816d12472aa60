/*
 * oedg.h -- C ABI of the MI355X (gfx950) BP RI-OEDG stage library.
 *
 * One SSP-RK3 stage of the bound-preserving, rotation-invariant
 * oscillation-eliminating discontinuous Galerkin scheme of Ding, Cui and Wu
 * (arXiv 2409.09620) for the 2D Euler equations on triangles, degree k = 1, 2:
 *   - the semi-discrete DG operator with the Lax-Friedrichs flux
 *     (eq. DGSystem:Dis, eq. fluxLF) and the SSP-RK3 combination (eq. RKTime);
 *   - the RIOE filter (eq. oe:sys with the coefficients of eqs. oe:sysdelta2,
 *     RIOESys:CoefM/Coef1/Coef2, OEScalar:beta/Coef2, normalised by eq. normOmg);
 *   - the Zhang-Shu-type BP limiter at the nodes of the optimal convex
 *     decomposition (Sec. 4.4, eqs. 1944/1981; nodes from eqs. 1040 and 1139);
 *   - the max wave speed (eq. 1250) and the optimal BP time step
 *     Delta t = C_SSP / alpha * min_K C^DCW_{K,k} |K| (Sec. 5, eqs. 1692, 1713).
 *
 * Conventions
 *   - Every call returns a dg_status; nothing throws or aborts.  The first error
 *     of a context is kept (dg_last_error) and later calls return it.
 *   - A context is bound to one HIP device and one stream and is NOT thread-safe.
 *     All device work is ordered on that stream.  Calls that return host data
 *     (dg_readback, dg_diag, dg_step_to, dg_step with dt_out) synchronise it.
 *   - Host arrays passed in are copied; the library never keeps host pointers.
 *   - Modal coefficients use the layout [var rho, m1, m2, E][mode l][cell] in
 *     float64, l = 0..L_k with L_1 = 2, L_2 = 5 and the basis of eq. basisfunc.
 *   - Device memory: the library allocates its buffers unless the caller binds a
 *     workspace (dg_bind_workspace) large enough for the mesh, which the caller
 *     owns and must keep alive until dg_destroy.
 */
#ifndef OEDG_H
#define OEDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_ctx dg_ctx;

typedef enum {
    DG_OK = 0,
    DG_E_ARG = -1,     /* invalid argument (null pointer, bad size, bad flag) */
    DG_E_MESH = -2,    /* invalid mesh (bad vertex id, zero area, an edge shared by >2 cells, no cells) */
    DG_E_NOMEM = -3,   /* device or host allocation failed, or bound workspace too small */
    DG_E_HIP = -4,     /* a HIP runtime call failed */
    DG_E_BOUNDS = -5,  /* a cell average left the admissible set (rho <= 0 or rho e <= 0) */
    DG_E_STATE = -6    /* call out of order (e.g. dg_stage before dg_init) */
} dg_status;

enum { DG_OE_RI = 0, DG_OE_CW = 1 };           /* rotation-invariant (Sec. 3.3) or component-wise (Sec. 3.2) */
/* Arithmetic of the stage (Sec. 6 runs everything in FP64; the mixed form is this
 * library's option).  DG_PREC_FP64: all of it in FP64.  DG_PREC_MIXED: cell
 * averages stored, updated and reduced in FP64; modes >= 1 stored in FP32 and the
 * volume/surface quadrature and OE filter in FP32; the BP limiter (point values,
 * theta, internal energy) and the max wave speed in FP64.  In the mixed form the
 * limiter's theta targets the floors plus a bound of the FP32 rounding of the
 * scaled modes, and the stored coefficients are re-checked: a cell whose stored
 * state would fall below half a floor at a node keeps only its average
 * (counted in dg_diag_t.n_flat).  Every limiter node of every stored state then
 * has rho >= eps_1/2 > 0 and rho e >= eps_2/2 > 0, evaluated in FP64.  The host
 * arrays of dg_init/dg_readback/dg_read_state stay FP64 in both forms (modes >= 1
 * are rounded to nearest FP32 on input). */
enum { DG_PREC_FP64 = 0, DG_PREC_MIXED = 1 };

/* Convex decomposition behind the BP limiter and the time step (Sec. 6 compares
 * the two).  DG_DECOMP_DCW: the optimal decomposition (Sec. 4.3): limiter nodes
 * are the 3Q edge Gauss points plus the P1 vertices opposite the two longest
 * edges (eq. 1944) or the two P2 internal nodes (eq. 1139), and
 * Delta t = C_SSP/alpha min_K C^DCW_{K,k}|K| (eqs. 1692, 1713).  DG_DECOMP_ZXS: the
 * classical Zhang-Xia-Shu decomposition (Sec. 4.2): the limiter takes the edge
 * Gauss points and, for P2, the vector u* = (ubar - sum_i w_i sum_nu w_nu
 * u(x_i,nu)) / (1 - sum_i w_i) with w_i = 1/9 (classical branch of Sec. 4.4; its
 * energy bound is E(u*)); C^ZXS_{K,k} = 1/(9 lbar_K) (P1), 1/(27 lbar_K) (P2),
 * lbar_K the mean edge length (remarks after eqs. 1692 and 1713). */
enum { DG_DECOMP_DCW = 0, DG_DECOMP_ZXS = 1 };

/* Form of the P2 limiter with the optimal decomposition (Sec. 4.4).
 * DG_LIMITER_NODES: the minima run over the 3Q edge Gauss points and both internal
 * nodes of eq. 1139, so the limited state is admissible at every node of the
 * decomposition.  DG_LIMITER_USTAR: Sec. 4.4's own form, the edge Gauss points and
 * the vector u* = (ubar - sum_i w_i sum_nu w_nu u(x_i,nu)) / (1 - sum_i w_i) with
 * the optimal edge weights w_i; u* is the mean of the two internal nodes, and
 * rho e(u*) is the energy bound.  It scales the modes no more than the node form
 * in each of its two steps.  P1 (eq. 1944) and the classical decomposition
 * ignore the setting. */
enum { DG_LIMITER_NODES = 0, DG_LIMITER_USTAR = 1 };

/* Boundary tags of unmatched edges (dg_mesh_upload's edge_bc).  Transmissive:
 * the exterior trace equals the interior one.  Reflective: the interior trace
 * with its normal momentum reversed, m - 2 (m.n) n.  The OE jump is zero on every
 * boundary edge and the wave speed uses the interior trace. */
enum { DG_BC_TRANSMISSIVE = 0, DG_BC_REFLECTIVE = 1 };

typedef struct {
    int k;             /* polynomial degree, 1 or 2 */
    double gamma;      /* adiabatic index (1.4 in the paper's Euler tests) */
    double c_ssp;      /* SSP coefficient of the RK3 scheme (1) */
    int oe_enable;     /* 1: apply the OE filter after every stage */
    int oe_mode;       /* DG_OE_RI or DG_OE_CW */
    int bp_enable;     /* 1: apply the BP limiter after every stage and at init */
    int precision;     /* DG_PREC_FP64 or DG_PREC_MIXED */
    int max_restarts;  /* retries of a step whose stage leaves the admissible set (8) */
    int decomposition; /* DG_DECOMP_DCW or DG_DECOMP_ZXS */
    int limiter_form;  /* DG_LIMITER_NODES or DG_LIMITER_USTAR */
} dg_config;

/* Fills *cfg with the defaults: k = 2, gamma = 1.4, c_ssp = 1, OE on (RI), BP on, FP64,
 * max_restarts = 8, the optimal decomposition (DG_DECOMP_DCW) with the node-form
 * limiter (DG_LIMITER_NODES).
 *
 * Step restarts (with the BP limiter on).  The BP time step bounds Delta t by the
 * wave speed of u^n (Sec. 5), while each stage's LF flux uses its own input's
 * speed; when a later stage's speed exceeds the step's, positivity of the averages
 * is no longer guaranteed for that stage.  A stage whose averages leave the
 * admissible set (rho <= 0 or rho e <= 0; the OE filter and the limiter keep the
 * averages, so this is decided in the residual pass) ends the attempt: the rest
 * of the step does nothing and u^n stays untouched; the step's last kernel then
 * halves Delta t and the next step launch retries it.  After max_restarts retries
 * of one step the run stops (DG_E_BOUNDS from the polling calls). */
void dg_config_default(dg_config* cfg);

/* Creates a context on HIP device `hip_device`.  `hip_stream` is a hipStream_t
 * owned by the caller (may be NULL: the null stream is used).  hip_device =
 * DG_HOST_ONLY gives a context without a device: dg_mesh_upload builds the host
 * tables (readable with dg_mesh_tables) and every device call returns DG_E_STATE. */
#define DG_HOST_ONLY (-1)
dg_status dg_create(dg_ctx** out, int hip_device, void* hip_stream);

/* Device bytes the library needs for a mesh of n_cell cells at degree k (enough
 * for either precision).  DG_E_ARG beyond DG_MAX_CELLS(k). */
dg_status dg_workspace_bytes(int32_t n_cell, int k, size_t* bytes);

/* Hands the library caller-owned device memory (at least dg_workspace_bytes),
 * used by the next dg_mesh_upload instead of its own allocation. */
dg_status dg_bind_workspace(dg_ctx* ctx, void* dev_ptr, size_t bytes);

/* Largest mesh at degree k: the kernels address a state buffer (4 variables x
 * (k+1)(k+2)/2 modes x n_cell doubles) with 32-bit byte offsets, so it stays
 * below 4 GiB: 44,739,242 cells at P1, 22,369,621 at P2. */
#define DG_MAX_CELLS(k) ((int32_t)(0xffffffffu / (32u * (unsigned)(((k) + 1) * ((k) + 2) / 2))))

/* Uploads a mesh and builds, on the host, what the paper's notation fixes
 * (Sec. 2 and Sec. 4.3): counter-clockwise orientation, the edge table (local
 * edge i is opposite local vertex i and runs from vertex i+1 to vertex i+2; the
 * neighbour across it and its local edge), per-cell geometry, the optimal
 * convex decomposition's limiter nodes and min_K C^DCW_{K,k}|K|.
 *   xy       host, 2*n_vert doubles (x, y per vertex)
 *   tri      host, 3*n_cell vertex ids (any orientation)
 *   cell_xy  host, 6*n_cell doubles or NULL: per-cell vertex coordinates used for
 *            the geometry instead of xy[tri] (periodic meshes: unwrapped images)
 *   edge_bc  host, 3*n_cell ints or NULL (all transmissive): edge_bc[3c+i] tags
 *            the edge of cell c opposite its input vertex i, DG_BC_TRANSMISSIVE
 *            or DG_BC_REFLECTIVE; entries of edges shared by two cells are
 *            ignored (a cell given clockwise is oriented by swapping its
 *            vertices 1 and 2, and its tags move with them)
 *   k        degree (1 or 2) the decomposition and the buffers are built for;
 *            dg_init must be called with the same degree
 * Errors: DG_E_ARG (also n_cell > DG_MAX_CELLS(k)), DG_E_MESH (the context is then
 * unusable), DG_E_NOMEM, DG_E_HIP. */
dg_status dg_mesh_upload(dg_ctx* ctx, int k, int32_t n_vert, const double* xy, int32_t n_cell,
                         const int32_t* tri, const double* cell_xy, const int32_t* edge_bc);

/* Host copies of the mesh tables built by dg_mesh_upload (any pointer may be NULL):
 * tri 3*n_cell (oriented), nbr 3*n_cell (-1 on the boundary), nbe 3*n_cell
 * (neighbour's local edge), perm 3*n_cell (local edges by decreasing length,
 * stable), node_ref 4*n_cell (reference coordinates (xi, eta) of the two extra
 * limiter points: P1 the vertices opposite the two longest edges (eq. 1944),
 * P2 the two internal nodes of eq. 1139), ck n_cell (C^DCW_{K,k}|K|), minck.  The
 * classical decomposition's C^ZXS_{K,k}|K| is fixed by the lengths and areas. */
dg_status dg_mesh_tables(dg_ctx* ctx, int32_t* tri, int32_t* nbr, int32_t* nbe, int32_t* perm,
                         double* node_ref, double* ck, double* minck);

/* Sets the configuration and the initial state u^0 (host, modal, layout above),
 * applies the BP limiter (no OE), computes alpha^0 and Delta t^0.  t = 0. */
dg_status dg_init(dg_ctx* ctx, const dg_config* cfg, const double* u0_modal);

/* As dg_init, with the state projected on the device from a named problem:
 * kind 0 isentropic vortex [x0,y0,eps,rho,u,v,p]; 1 four quadrants
 * [xc,yc,(rho,u,v,p) x 4]; 2 blast [E_total,p_amb,rho,origin_vertex]; 3 two
 * states [px,py,nx,ny,(rho,u,v,p)_L,(rho,u,v,p)_R].  L2 projection with the
 * 12-point rule of tab:6th; the blast sets cell averages only. */
dg_status dg_init_problem(dg_ctx* ctx, const dg_config* cfg, int kind, const double* params,
                          int n_params);

/* One stage s = 0, 1, 2 of the current step: residual + SSP combination, the
 * domain reductions, the OE filter, the BP limiter and the max wave speed of
 * the result.  Stage 2 also advances t and the step count and sets the next
 * Delta t.  No host synchronisation. */
dg_status dg_stage(dg_ctx* ctx, int s);

/* dg_stage without device memory of its own, for callers that cannot allocate
 * (code under HIP graph capture, serving loops that forbid allocation): the same
 * kernels in the same order, with the per-workgroup partial records of the two
 * domain reductions in a device array of the library instead of the context's
 * workspace.  Results are bit-identical to dg_stage.
 *   The array holds the records of at most 4096 workgroups per pass (26 doubles
 * each, 851,968 bytes per GPU); each GPU the library runs on keeps its own copy
 * until the process ends.  Its address is looked up once per device, at
 * dg_create (or at the first call on the device).  The passes size their grids
 * by occupancy, at most 4096 workgroups, so every mesh fits; a grid beyond the
 * array returns DG_E_ARG.  Every workgroup writes its whole record before the
 * reduction reads it (the passes of a step skipped after an inadmissible stage
 * write none, and their reductions then use none of what they read), so nothing
 * needs clearing between calls.
 *   The call performs no hipMalloc, hipFree or other allocation and does not
 * synchronise.  All calls on one GPU share its array: calls that overlap on
 * that GPU (other streams, other host threads, other contexts) race and give
 * wrong results; calls ordered on one stream do not.
 * Errors: as dg_stage; DG_E_HIP if the array's address cannot be obtained. */
dg_status dg_stage_noalloc(dg_ctx* ctx, int s);

/* One full step (three stages).  If dt_out is not NULL the stream is
 * synchronised and the step's Delta t is written there. */
dg_status dg_step(dg_ctx* ctx, double* dt_out);

/* Steps until t reaches t_end (the last step is shortened to land on it) or
 * max_steps steps were completed (retried attempts do not count).  Synchronises
 * every few steps to poll. */
dg_status dg_step_to(dg_ctx* ctx, double t_end, int64_t max_steps, int64_t* steps_done);

/* Copies u^n (host, modal, layout above) and the time and step count.  After a
 * DG_E_BOUNDS stop it still copies (the u^n the failed step started from) and
 * returns DG_E_BOUNDS. */
dg_status dg_readback(dg_ctx* ctx, double* u_modal, double* t, int64_t* step);

/* Copies an internal state buffer: which = 0 u^n, 1 last stage output,
 * 2 last pre-filter state (before OE and limiter). */
dg_status dg_read_state(dg_ctx* ctx, int which, double* u_modal);

typedef struct {
    double t, dt, alpha;          /* time, current step, LF viscosity of u^n */
    int64_t step;
    int64_t n_limited;            /* cell-stages where the limiter scaled modes */
    int64_t n_bad;                /* cell averages outside the admissible set */
    int64_t n_cfl_excursions;     /* stages whose alpha exceeded the step's alpha */
    double ubar[4];               /* domain averages of the last pre-filter state */
    double nrm[4];                /* ||u - ubar||_inf per variable (eq. normOmg) */
    double nrm_m;                 /* ||| m - mbar |||_inf (vector norm) */
    int active;                   /* 0 once t has reached the last t_end */
    int64_t n_flat;               /* DG_PREC_MIXED: cell-stages reset to their average by the
                                     check of the stored (FP32-rounded) coefficients */
    int64_t n_restarts;           /* steps retried with half the time step */
    double alpha_stage;           /* LF viscosity of the next stage's input (eq. 1250):
                                     alpha of u^n before stage 0, of the last stage
                                     output after stages 0 and 1 */
    double min_rho_node;          /* min density over every limiter node (Sec. 4.4) of
                                     the last stage output, evaluated in FP64 */
    double min_p_node;            /* min pressure there */
} dg_diag_t;

/* Diagnostics of the context (synchronises). */
dg_status dg_diag(dg_ctx* ctx, dg_diag_t* out);

/* Kernel timing with HIP events recorded on the context's stream around every
 * stage kernel launch (a few microseconds of overhead per launch).
 * dg_profile_enable(ctx, 1) starts recording; dg_profile_read synchronises, adds
 * the elapsed times since the last read into ms[k] and the launch counts into
 * launches[k] for k = 0 residual pass, 1 filter pass, and restarts the
 * accumulation.  Both arrays have DG_PROFILE_KERNELS entries. */
#define DG_PROFILE_KERNELS 2
dg_status dg_profile_enable(dg_ctx* ctx, int enable);
dg_status dg_profile_read(dg_ctx* ctx, double* ms, int64_t* launches);

/* Sets the stop time of a context's run without stepping (as dg_step_to does
 * before it steps): the last step is shortened to land on t_end and the context
 * turns inactive once t reaches it.  Stream-ordered, no synchronisation.  Used
 * to give the members of a batch their own end times. */
dg_status dg_set_t_end(dg_ctx* ctx, double t_end);

/* ---------------------------------------------------------------------------
 * Batches: several initialised contexts on one device (meshes of any size,
 * degrees 1 and 2 mixed, one precision) stepped together, each pass of a
 * stage one persistent launch over all members of a degree (two launches on
 * parallel streams when both degrees are present; the method is per instance,
 * batching is this library's scheduling).  A chunk table cuts every member into
 * runs of 256-cell reduction groups, split into one contiguous range per XCD by
 * estimated cost; every group writes its own partial record and a
 * per-member finalize reduces them in a fixed order.  A member's result
 * therefore does not depend on the schedule or on the other members: it is the
 * same, bit for bit, as in a batch of its own (not as dg_step, whose
 * single-instance passes group the reductions differently, within round-off).
 * Each member keeps its own alpha, Delta t, t and t_end (dg_set_t_end); members
 * that reached their t_end are skipped.  The batch borrows the contexts: they
 * must outlive it, must not be stepped on other streams while it runs, and
 * re-initialising one (dg_init, dg_init_problem, dg_mesh_upload) makes the
 * batch return DG_E_STATE.  The batch allocates its own device memory (stage
 * arguments, chunk table, 26 doubles per 256 cells of partial records) and,
 * with both degrees present, a second stream and two events. */
typedef struct dg_batch dg_batch;

/* Builds a batch of n contexts on hip_stream (may be NULL).  Errors: DG_E_ARG
 * (n <= 0, a context listed twice, different devices or precisions),
 * DG_E_STATE (a context not initialised or failed), DG_E_NOMEM, DG_E_HIP.  On
 * DG_E_NOMEM/DG_E_HIP *out is set and must still be destroyed. */
dg_status dg_batch_create(dg_batch** out, dg_ctx* const* ctxs, int n, void* hip_stream);

/* Schedule: chunk_groups reduction groups (256 cells each) per chunk, and the
 * pass grids at occupancy_pct percent of the resident workgroups. */
dg_status dg_batch_set_schedule(dg_batch* b, int chunk_groups, int occupancy_pct);
dg_status dg_batch_get_schedule(const dg_batch* b, int* chunk_groups, int* occupancy_pct, int* n_chunks,
                                int* grid /* 2: residual, filter; workgroups over both degrees' launches */);

/* Times stage 0 of the batch for chunk_groups in {1,2,4,8,16} and occupancy in
 * {100, 50} percent (reps timed runs each, after a warm-up), keeps the fastest
 * and returns it.  The members' states are unchanged: stage 0 only writes
 * scratch buffers, and their device scalars are restored.  Synchronises. */
dg_status dg_batch_autotune(dg_batch* b, int reps, int* chunk_groups, int* occupancy_pct, double* ms_stage);

/* n_steps SSP-RK3 steps of every active member (no synchronisation). */
dg_status dg_batch_step(dg_batch* b, int64_t n_steps);

/* Steps until no member is active or max_steps step launches were made (a
 * launch completes or retries each active member's step); polls every
 * few steps.  DG_E_BOUNDS if a member's cell average left the admissible set. */
dg_status dg_batch_run(dg_batch* b, int64_t max_steps, int64_t* steps_done);

/* Synchronises and reports the number of active members and, if status is not
 * NULL, {active, error, t, step} of member i in status[4 i .. 4 i + 3]. */
dg_status dg_batch_status(dg_batch* b, int* n_active, double* status);

/* Host-only planning (no device): the chunk table of n_inst instances with
 * n_cell[i] cells at degree k[i] and chunk_groups groups per chunk.  Writes the
 * number of chunks to *n_chunks and, when chunks is not NULL (capacity
 * max_chunks), chunk c as (instance, first group, end group) in chunks[3c..];
 * split (9 ints, may be NULL) receives the chunk range boundaries per XCD. */
dg_status dg_plan_chunks(int n_inst, const int32_t* n_cell, const int* k, int chunk_groups, int32_t* chunks,
                         int max_chunks, int* n_chunks, int32_t* split);

const char* dg_batch_last_error(const dg_batch* b);
void dg_batch_destroy(dg_batch* b);

/* Number of cells, degree and modes of the uploaded mesh. */
dg_status dg_sizes(dg_ctx* ctx, int32_t* n_cell, int* k, int* n_modes);

/* Last error message of the context (never NULL). */
const char* dg_last_error(const dg_ctx* ctx);

/* Frees the context and the memory the library allocated. */
void dg_destroy(dg_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* OEDG_H */
