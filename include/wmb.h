/*
 * wmb.h -- C ABI of the MI355X (gfx950) library that advances batches of
 * ghosted Cartesian patches of 3D ideal MHD by the MHDTVD CTU+CT scheme of
 * Mendygral et al. 2017 (WOMBAT), Sect. 5.2 ("MHD in Three Dimensions",
 * Steps 1-11) with the MHDTVD flux of Appendix A.
 *
 * The verbs follow the paper's statement of the problem (Sect. 2.1, 4.1): a
 * world grid (periodic, or with outflow ends as in the shock tubes of Sect. 6)
 * cut into patches with their own boundary zones; ghost zones filled between
 * patches; a global CFL reduction for dt (Sect. 4.1.1); a solver that updates
 * the patch arrays; state read back.
 *
 * Conventions shared by every entry point
 *   - Return value: WMB_OK (0) or a negative WMB_E* code.  Nothing aborts or
 *     throws across this boundary.  wmb_last_error() gives a message for the
 *     last failure on a context.
 *   - Ownership: the caller owns the device pool (one allocation of at least
 *     wmb_pool_bytes() bytes, e.g. a torch uint8 tensor) and the HIP stream;
 *     both must outlive the context, which never frees them.  The library owns
 *     the context, its small device tables (descriptors, work lists, dt and
 *     reduction scratch) and its captured graphs; wmb_destroy frees them.
 *   - Host arrays belong to the caller.  wmb_set_state / wmb_get_state /
 *     wmb_compute_dt(out != NULL) / wmb_diagnostics are synchronous on the
 *     stream; wmb_fill_ghosts, wmb_advance and wmb_run_steps only enqueue.
 *   - One context is used by one host thread at a time.
 *   - Layout of host state arrays (double, C order): q is 8 x nz x ny x nx in
 *     the paper's component order (rho, rho vx, rho vy, rho vz, Bx, By, Bz, E)
 *     (Sect. 5, 1D conservative form); b is 3 x nz x ny x nx, where b[a] at
 *     zone (i,j,k) is the face-centred field component a on the zone's LEFT
 *     face along a (x_{i-1/2} for a = x, and so on).  Units carry no 4 pi.
 *   - Device layout (inside the pool): per patch, structure of arrays over
 *     the ghosted box (n+2g)^3, x fastest, FP32 or FP64 by precision.
 */
#ifndef WMB_H
#define WMB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WMB_OK 0
#define WMB_EINVAL (-1) /* bad argument or inconsistent patch table */
#define WMB_ENOMEM (-2) /* host or library-owned device allocation failed */
#define WMB_EHIP (-3)   /* a HIP runtime call failed (message in last_error) */
#define WMB_ESTATE (-4) /* non-finite input, rho <= 0 or P <= 0 */
#define WMB_ECFL (-5)   /* dt above the CFL limit */
#define WMB_ESIZE (-6)  /* pool smaller than wmb_pool_bytes */
#define WMB_EORDER (-7) /* call out of sequence (e.g. advance before init) */

#define WMB_FP64 0 /* all stages in double */
#define WMB_FP32 1 /* sweeps and CT in float; dt, floors, diagnostics in double */

typedef struct wmb_params {
    double gamma;        /* adiabatic index (Sect. 5) */
    double cfl;          /* Courant number of the dt reduction */
    double eps[7];       /* entropy-fix epsilon_k of Q_k (Appendix A), 0 <= eps < 0.5,
                            waves in ascending order v-cf, v-ca, v-cs, v, v+cs, v+ca, v+cf */
    double limiter_beta; /* Sweby limiter parameter in [1, 2] (Appendix A) */
    double rho_floor;    /* density floor (Appendix A, last paragraph) */
    double p_floor;      /* pressure floor */
    double dx[3];        /* zone widths along x, y, z */
    double degen_tol;    /* degeneracy threshold of the eigenvectors (e.g. 1e-12) */
    int32_t ghost;       /* ghost width g, >= 4 (the paper uses 5, Sect. 5.1) */
    int32_t precision;   /* WMB_FP64 or WMB_FP32 */
    double rho_protect;  /* protection floors (Appendix A, last paragraph): a face */
    double p_protect;    /* whose Roe sound speed squared is not positive, or one of
                            whose six Roe-fan intermediate states u_L + sum_{k<m}
                            alpha_k R_k has rho < rho_protect or P < p_protect,
                            takes the HLL flux instead of the MHDTVD flux (and
                            contributes no g-tilde to its zones' limiters); both 0
                            (the default) switch the protection off */
    int32_t dt_lag;      /* 0 (default): dt of step n from the state q^n.  1: from
                            q^(n-1), the state one step earlier (the first step of
                            a run from q^0): the paper delays the dt reduction by
                            one step to overlap it with work (Sect. 4.1.1) */
    int32_t scratch_groups; /* 0 or 1 (default): every patch has its own space for
                            the step's intermediates (51 words a ghosted zone
                            beside its 22 words of state).  G = 2..64: the
                            patches are dealt, whole x-rows at a time, to G
                            groups whose steps run one after another and share
                            one space for the intermediates, sized for the
                            largest group: the pool takes 22 + 51/G words a
                            zone (at G = 4, 34.75).  The step schedule is then
                            fixed to those groups (wmb_set_schedule) */
} wmb_params;

typedef struct wmb_patch_desc {
    int32_t n[3];      /* interior zones along x, y, z (each >= ghost) */
    int32_t nbr[27];   /* patch id at offset (dz,dy,dx) in {-1,0,1}^3, index
                          9(dz+1) + 3(dy+1) + (dx+1); the caller resolves
                          periodic wrap; nbr[13] is the patch itself; -1 where
                          the offset leaves the domain (an outflow boundary:
                          zero-gradient ghosts).  Face neighbours must share
                          the face extent. */
    int64_t origin[3]; /* global zone offset (diagnostics only) */
} wmb_patch_desc;

typedef struct wmb_ctx wmb_ctx;

/* Create a context.  Validates p (gamma > 1, cfl in (0,1], ghost >= 4,
   dx > 0, precision known, protection floors >= 0, dt_lag 0 or 1,
   scratch_groups 0..64).  *out receives the context. */
int wmb_create(const wmb_params *p, wmb_ctx **out);

/* Device bytes the caller must provide for npatch patches: each patch's
   state region (two state copies, 11 words per stored zone each), then the
   space for the step's intermediates (51 words per stored zone: a slot per
   patch, or with scratch groups a slot per patch of the largest group). */
int wmb_pool_bytes(const wmb_params *p, int32_t npatch, const wmb_patch_desc *d, uint64_t *bytes);

/* Bind the patches to the caller's device pool and stream (hipStream_t, NULL
   = default stream).  Checks the neighbour table (face extents agree, the
   neighbour of my neighbour is me; every interior edge at least the ghost
   width; a patch's intermediates, 51 words per ghosted zone, at most 4 GiB) and
   builds the launch plans.  The pool's
   contents are undefined until wmb_set_state has been called for every
   patch.  WMB_ESIZE if pool_bytes < wmb_pool_bytes. */
int wmb_init_patches(wmb_ctx *c, int32_t npatch, const wmb_patch_desc *d, void *dev_pool,
                     uint64_t pool_bytes, void *hip_stream);

/* Upload one patch's interior state (host arrays, layout above).  Rounds to
   FP32 in FP32 mode.  WMB_ESTATE if any value is non-finite, rho <= 0, or the
   pressure (from E with the zone-centred field) is <= 0.  Along an axis whose
   +side is a domain boundary the patch owns its right face n (no neighbour
   holds it): it starts as a copy of face n-1.  On a frozen patch (see
   wmb_set_active) the call also refreshes every ghost and makes both internal
   state copies equal. */
int wmb_set_state(wmb_ctx *c, int32_t patch, const double *q, const double *b);

/* Read one patch's interior state (and its own left faces) back to host
   double arrays, same layout as wmb_set_state. */
int wmb_get_state(wmb_ctx *c, int32_t patch, double *q, double *b);

/* Read the whole ghosted box of one patch: q is 8 x Nz x Ny x Nx, b is
   3 x Nz x Ny x Nx with N = n + 2 ghost (test hook for the ghost exchange). */
int wmb_get_stored(wmb_ctx *c, int32_t patch, double *q, double *b);

/* Enqueue the ghost exchange (Sect. 4.1, local patch copies): every ghost
   zone and ghost face of every patch becomes a copy of the neighbour's
   interior value covering it; a patch's right-boundary face is the
   neighbour's own left face.  Beyond a domain boundary (-1 in the table) a
   ghost zone copies the nearest interior zone (its index clamped into
   [0, n-1] along that axis) and the face component normal to the boundary
   copies the boundary face (index clamped into [0, n]); edges and corners
   compose the clamps axis by axis.  Bitwise copies. */
int wmb_fill_ghosts(wmb_ctx *c);

/* CFL reduction in FP64 over all interior zones of the active patches:
   dt = cfl * min_{zones, d} dx_d / (|v_d| + c_f,d), with c_f,d the fast speed
   (Sect. 5) taking B_d as the longitudinal field.  The result stays in device
   memory for wmb_advance(c, 0) / wmb_run_steps; if dt_out != NULL it is also
   copied to the host (synchronising the stream).  With dt_lag = 1 the steps
   of wmb_run_steps use the maximum of the state one step earlier; a run
   whose state was set from the host, or follows this call, starts again
   from the current state. */
int wmb_compute_dt(wmb_ctx *c, double *dt_out);

/* One CTU+CT step (Sect. 5.2, Steps 1-11) of every patch.  Ghosts must be
   current.  dt > 0: use this dt (the call checks it against the CFL limit of
   the current state and returns WMB_ECFL if it is larger by more than 1e-12
   relative; this check synchronises and reduces the current state afresh:
   with dt_lag = 1 the maximum a step folds in belongs to the state before,
   and lagged steps after this call start again from the current state).
   dt <= 0: use the device-resident dt of the last wmb_compute_dt.  Floors
   (rho_floor, p_floor) are applied in FP64 and counted.  The step also writes the new state of the first and last
   ghost-width zones of every interior row into the x-neighbours' ghosts (the
   x part of the next ghost exchange; at a domain boundary the patch's own
   x-ghosts by zero gradient; next to a frozen neighbour it copies that
   neighbour's zones into its own x-ghosts instead); other ghosts are left to
   wmb_fill_ghosts.  Frozen patches are not advanced. */
int wmb_advance(wmb_ctx *c, double dt);

/* nsteps x (fill ghosts, compute dt, advance) with dt kept on the device,
   replayed from a captured HIP graph (captured on the first call).  The
   graph's ghost exchange runs the y and z passes only (the step before wrote
   the x-ghosts), on a branch of its own beside the part of the Step-1 x sweep
   whose pencils have interior transverse coordinates (the overlap of
   exchange and interior work of Sect. 4); the three sweeps of each stage
   run as concurrent branches (library-owned streams, default priority),
   except that the fused corrector is followed by the z sweep that reads its
   records; the
   x pass is enqueued first when the state was set since.  Results are
   bitwise those of the eager calls.  Enqueue only; this is the timed call. */
int wmb_run_steps(wmb_ctx *c, int32_t nsteps);

/* FP64 diagnostics over all interiors: totals[8] = sum over zones of q times
   the zone volume; max_divb_raw = max |div b| with div b = sum_d (b_d(+) -
   b_d(-)) / dx_d; max_divb_norm = max_divb_raw * min(dx) / B_rms; n_floored =
   floor activations since wmb_init_patches; n_protected = faces that took the
   HLL flux since wmb_init_patches (every computed face of every stage,
   including faces in the ghost halo).  Any output pointer may be NULL. */
int wmb_diagnostics(wmb_ctx *c, double totals[8], double *max_divb_norm, double *max_divb_raw,
                    int64_t *n_floored, int64_t *n_protected);

/* Allocation-free variant of wmb_diagnostics, for callers that cannot
   allocate (code under HIP graph capture, tight serving loops, harnesses
   that forbid allocation): enqueues the same kernels on the context's stream
   and writes 12 doubles to dev_out, a caller-owned device array: totals[0..7],
   max_divb_norm, max_divb_raw, n_floored, n_protected (counts as exact
   doubles), bitwise what wmb_diagnostics returns for the same state.  It
   allocates nothing and does not synchronise: the per-record partial sums go
   to a static device array of 32768 records (5 MiB) that each GPU the
   library runs on holds until the process ends.  Every call on a GPU shares
   that array: calls that overlap on one GPU (contexts on several streams)
   race; each call rewrites every record it reads, so nothing has to be
   cleared between calls.  WMB_ESIZE if the batch needs more than 32768
   records (one per started run of 32768 interior zones of a patch),
   WMB_EINVAL for a NULL dev_out. */
int wmb_diagnostics_noalloc(wmb_ctx *c, double *dev_out);

/* Test hook: copy an intermediate of the last step of one patch over the
   ghosted box, widened to double, in this layout: stage 1 Step-1 fluxes
   (3 x 8 x vol, lab component order, B_par row 0), 3 b^{n+1/2} (3 x vol),
   5 Step-6/7 fluxes (3 x 8 x vol), 6 Step-9 edge EMFs (3 x vol; only after
   a step run with wmb_keep_stages on, else WMB_ESTATE).  Values outside the
   ranges the step needs are unspecified; with scratch groups only the
   patches of the last group hold their own.  Other stages (the Step-3 edges are
   overwritten by Step 9) give WMB_EINVAL.  Synchronous. */
int wmb_debug_stage(wmb_ctx *c, int32_t patch, int32_t stage, double *out);

/* Search the shape of the directional sweeps for every group of patches
   with the same edge along the sweep axis, timing each candidate `reps`
   times on the device, and keep the fastest.  A shape W > 0 is the LDS
   pencil form with W pencils a block (every thread one zone of a pencil);
   W < 0, for the y and z sweeps only, is the marching form with -W pencils
   a block (every thread walks one whole pencil, consecutive lanes on
   consecutive x, the face data carried in registers); in FP32, W = -(w + 512)
   selects for the corrector sweeps (Steps 6-7) the marching variant that
   issues the next zone's loads one zone ahead (w pencils a block; more
   registers, half the waves).  The choice never
   changes results (both forms compute every face with the same
   arithmetic).  It then times whole graph-replayed steps with the x and y
   correctors fused into one launch (bands of 6, 9, 12 or 18 rows, where
   the blocks fit, each with three shapes of the z corrector that reads the
   records it stores) against the separate sweeps, and the tiles of Steps 3-4
   (the widest tile along x: 40, 20 or 13 zones, 256 zones a plane) and of
   Steps 8-11 (256 or, in FP32, 512 zones a plane) with either Steps 8-11
   launch; none of these changes results either.  The
   interior state is unchanged; ghosts are refreshed and the step
   intermediates overwritten.  Invalidates the captured graphs.  The choice
   is kept for the life of the process under a key of the device
   architecture, the precision, the ghost width, the limiter and protection
   variants and the patch extents with their counts: a later call with the
   same key (on any context) applies it without timing.  reps < 0 times
   anyway, with -reps repetitions, and replaces the kept choice.  If chosen
   != NULL it receives quadruples (stage, axis, edge, shape) -- the sweep
   groups, then (3, 0, 0, Steps 3-4 tile width), (4, 0, 0, Steps 8-11
   tile zones), (5, 0, 0, Steps 8-11 launch) and (6, 0, 0, fused x/y
   corrector band rows, 0 for separate sweeps) -- up to nchosen ints,
   0-terminated when shorter.
   Synchronous. */
int wmb_autotune(wmb_ctx *c, int32_t reps, int32_t *chosen, int32_t nchosen);

/* Set the shapes of sweep groups directly: quads of (stage 1|2, axis 0..2,
   edge along the axis, shape), n ints in total (a multiple of 4), as
   returned by wmb_autotune (shape > 0: pencil form with that many pencils a
   block; shape < 0: marching form, y and z only, with -shape pencils a
   block, at most 256, or -(w + 512) for the FP32 corrector with the loads
   one zone ahead).  Groups not named keep their shape.  WMB_EINVAL if a
   pencil shape exceeds 1024 threads or 64 KiB of LDS, or a marching shape
   is asked for x or beyond 256.  Invalidates the captured graphs.  The
   defaults are the marching form (64 pencils a block) for the y and z
   sweeps in FP32 and the pencil form elsewhere.  Tile entries: (3, 0, 0, w)
   sets the widest Steps 3-4 tile along x to w zones (4..40, default 40);
   (4, 0, 0, z) the zones of a Steps 8-11 tile plane (256, or 512 in FP32;
   the default is the one that leaves fewer threads idle); (5, 0, 0, m) the
   Steps 8-11 launch: m = 0 one block a tile (the default), m = 1 a
   persistent grid whose blocks take the tiles of their XCD's queue from an
   atomic counter; (6, 0, 0, r) the corrector (Steps 5-7): r = 0 three
   separate sweeps (the FP64 default), r > 0 (the FP32 default: 9, or 6
   where those blocks do not fit) one fused launch for x and y whose
   blocks each take one z-plane of a patch and a band of at most r rows
   along y, build the x, y and z predictor states of their zones from one
   block's loads, form the x and y faces and store the z predictor records
   in the z flux rows, which the z corrector sweep then reads instead of
   q^n and the Step-1 fluxes (bitwise the same fluxes; the y corrector
   groups' shapes are then unused, the z ones shape that sweep).  WMB_EINVAL
   if a block of (n_x + 6) x (r + 3) threads, for any x edge, exceeds 1024
   threads or 64 KiB of LDS (16 words a thread).  Every entry is checked
   before any is applied. */
int wmb_set_tuning(wmb_ctx *c, const int32_t *quads, int32_t n);

/* Schedule of the captured step (wmb_run_steps).  groups = 1 (the default):
   the three sweeps of each stage (the separate ones) run as concurrent
   branches and the y/z ghost exchange beside the interior part of the
   Step-1 x sweep.  groups =
   2..4: the patches are dealt, whole x-rows at a time, to that many groups,
   and each group runs its whole step (Steps 1-11) on a stream of its own
   after the exchange and dt, so that the memory-bound stages of one group
   overlap the sweeps of another (the paper's update engine works on
   patches in different stages at once, Sect. 4.1).  Results are bitwise
   the same under every schedule; wmb_advance and wmb_profile_step always
   run the stages one after another.  Invalidates the captured graphs.
   WMB_EINVAL outside 1..4. */
int wmb_set_schedule(wmb_ctx *c, int32_t groups);

/* Freeze (active = 0) or thaw (active != 0) one patch without rebuilding
   the launch plan or the captured graphs (Sect. 2.1: patches may become
   inactive, left out of the update, for load balancing and mesh
   refinement; here its pool memory stays reserved).  A frozen patch keeps
   its state: no kernel updates it, it adds nothing to the CFL maximum or to
   the floor and protection counters, and it serves its neighbours as fixed
   ghost data (its work items exit at once).  Its state then reads the same
   in both internal state copies, which freezing establishes by refreshing
   every ghost and copying the patch's stored box; wmb_set_state on a frozen
   patch does the same.  The face it shares with an active neighbour stays
   the frozen patch's.  Diagnostics still cover every present patch.  With
   every patch frozen the CFL maximum is empty: dt comes out +inf and steps
   change nothing.  All patches start active.  Asynchronous: the work (the
   ghost refresh, the copy and the patch-table entry) is enqueued on the
   library's stream, ordered before the next step.  The next call that
   steps (wmb_advance, wmb_run_steps, wmb_profile_step, wmb_autotune) plans
   the stage work lists again without the frozen patches, in place (it
   waits for the stream once): the graphs keep their buffers and grid sizes
   and stay valid.  WMB_EINVAL for a patch index out of range, WMB_EORDER
   for an absent patch. */
int wmb_set_active(wmb_ctx *c, int32_t patch, int32_t active);

/* Remove (present = 0) or add back (present != 0) one patch slot of the
   table given to wmb_init_patches, without rebuilding the launch plan or
   the captured graphs (Sect. 2.1: a domain allocates and frees patches, for
   load balancing and mesh refinement; here the slot's pool memory stays
   reserved, so the slots are the patches the domain may ever hold).  A
   removed slot leaves the domain: no kernel reads or writes it, the
   diagnostics leave it out, and its face neighbours see a domain boundary
   there (zero-gradient ghosts; edge and corner ghosts still arrive through
   the x, y, z order of the exchange).  Removal first refreshes every ghost,
   so the faces the slot shared with its neighbours keep their last values
   and become those neighbours' own boundary faces.  Adding a slot back links
   it to its face neighbours of the init table that are present, active;
   it brings the state the slot holds (set it with wmb_set_state before or
   after, before the next step).  Each patch owns the faces on its low sides
   (-x, -y, -z): the added slot's low faces replace its present neighbours'
   copies at the next exchange and its high faces take theirs, so div b is
   kept on the shared faces when the given state matches them.
   Asynchronous (the table entries are enqueued on the library's stream);
   the work lists are planned again as after wmb_set_active.  All slots
   start present.  WMB_EINVAL for a patch index out of range. */
int wmb_set_present(wmb_ctx *c, int32_t patch, int32_t present);

/* Debugging: with on != 0, later steps also store the Step-9 edge EMFs in
   device memory for wmb_debug_stage (the fused Steps 8-11 otherwise keep
   them on chip).  Default off.  Invalidates the captured graphs when it
   changes. */
int wmb_keep_stages(wmb_ctx *c, int32_t on);

/* Benchmark hook: enqueue one (fill ghosts, compute dt, advance) with the
   same launches the captured graph replays, with a HIP event recorded on the
   context's stream after each kernel class, wait for it, and store the
   duration in milliseconds of each class in ms[0 .. WMB_NCLASS-1], in this
   order: fill (3 passes), dt (finalize of the reduction that the previous
   update folded in), sweep x, y, z (Step 1, the x sweep also forming the
   Step-2 reference EMF), CT half (Steps 3-4 fused: edge EMFs and
   b^{n+1/2}), sweep x, y, z (Steps 5-7; with the fused corrector its launch
   counts as x, y is empty and z is the sweep from its records), update
   (Steps 8-11 fused:
   half-step EMF, edge EMFs, conservative and CT update, and the
   signal-speed maximum of the new state).  Advances the state by one step.
   Synchronous. */
#define WMB_NCLASS 10
int wmb_profile_step(wmb_ctx *c, double *ms, int32_t nclass);

/* Free the context, its tables and graphs (not the pool, not the stream).
   The streams the library uses besides the caller's (two for the concurrent
   branches of the step graph, and its own main stream when the caller passed
   NULL) are not destroyed but kept for later contexts on the same device:
   on ROCm 7, destroying a stream that took part in a graph capture before
   the memory its captured kernels used is freed keeps that memory from ever
   being freed, and the caller frees its pool after this call. */
int wmb_destroy(wmb_ctx *c);

/* Static message for an error code. */
const char *wmb_strerror(int code);

/* Message of the last failure on this context ("" if none). */
const char *wmb_last_error(const wmb_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* WMB_H */
