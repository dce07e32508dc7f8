/*
 * dcfmm.h -- C ABI of the MI355X (gfx950) diffusion-curve library.
 *
 * The library solves and renders diffusion curves with the hybrid BEM/BIEM
 * discretisation of Bang, Serkh, Stein and Jacobson (ACM TOG 42(6), 2023):
 * densities live at Gauss-Legendre nodes on cubic Bezier panels (Sec. 4.3,
 * 5.2), potentials are integrated over chord segments with closed forms
 * (App. D) scaled to the true arc length (App. A), and both the solve
 * (Alg. 3) and the render (Alg. 4) are accelerated by a 2D Laplace fast
 * multipole method on a non-uniform quadtree (App. E, Alg. 8).
 *
 * Conventions shared by every entry point
 *  - Curves: ctrl[c][k][xy], k = 0..3 control points, math axes (y up).
 *  - Colours: left_rgb/right_rgb[c][stop][rgb]; stop k sits at normalised
 *    arc length k/(n_stops-1); colour is linear in arc length between stops.
 *    The "+" side of a curve is the side its left normal (tangent rotated
 *    +90 degrees) points to, so u+ = left colour, u- = right colour
 *    (Sec. 5.3, Eq. int_S_dbnd_twoside).
 *  - Nodes are numbered curve-major, then panel, then GL node in increasing
 *    parameter: i = (c*P + p)*g + k, or i = panel*g + k for a scene made
 *    from a panel list (panels listed curve by curve, in order along each).
 *    Densities are [3][N] (channel-major).
 *  - Pixels: row r, column k of a W x H viewport with centre (cx, cy) and
 *    size (width, height) sit at x = cx - width/2 + (k+1/2) width/W,
 *    y = cy + height/2 - (r+1/2) height/H.  Images are [H][W][3], row 0 at
 *    the top.  Values are not clamped.
 *  - Ownership: the library copies every host input it is given; output
 *    buffers are owned by the caller.  "dev" pointers are device pointers on
 *    the current HIP device; "stream" is a hipStream_t (NULL = default).
 *    Calls that take a stream enqueue their kernels on it and return without
 *    waiting unless stated otherwise.
 *  - Errors: every int-returning call returns DC_OK (0) or a negative code;
 *    dc_last_error() returns a thread-local message for the last failure.
 *    No exception crosses the ABI.  A scene is not thread-safe: calls on one
 *    scene must not overlap.
 */
#ifndef DCFMM_H
#define DCFMM_H

#ifdef __cplusplus
extern "C" {
#endif

#define DC_OK 0
#define DC_ERR_INVALID (-1)        /* bad argument, NaN or degenerate input */
#define DC_ERR_OOM (-2)            /* device or host allocation failed */
#define DC_ERR_NOT_CONVERGED (-3)  /* GMRES hit max_iter; report filled */
#define DC_ERR_HIP (-4)            /* HIP runtime error; message kept */
#define DC_ERR_TIMEOUT (-5)        /* dc_server_wait: not done in time;
                                      render calls and server requests: an
                                      earlier render of the scene stalled
                                      on the device (a bounded wait of the
                                      render kernel ran out) and its images
                                      are incomplete */

#define DC_PREC_F64 0   /* everything in FP64 */
#define DC_PREC_F32 1   /* FP32 M2L, L2L, L2P, near field and P2L of
                           small charges; FP64 upward pass, stored
                           expansions, M2P, P2L of large charges and
                           near-singular chord pairs */
#define DC_METHOD_FMM 0
#define DC_METHOD_DIRECT 1   /* brute-force sum over every chord segment */
#define DC_OUT_F32 0
#define DC_OUT_F64 1
#define DC_P_MAX 63          /* largest expansion order supported */

typedef struct dc_scene_s* dc_scene;

/* Discretisation and quadtree of a scene.
 * panels_per_curve P, gl_per_panel g, segs_per_panel s (the same segments
 * are used for solution and evaluation, s = e, Sec. 9), leaf_max b (a box is
 * split while it holds more than b GL nodes; App. E.5), max_depth (<= 40),
 * domain = {xmin, ymin, xmax, ymax}: a rectangle the quadtree root must cover
 * besides the curves (every rendered pixel centre must lie in the root). */
typedef struct {
    int panels_per_curve;
    int gl_per_panel;
    int segs_per_panel;
    int leaf_max;
    int max_depth;
    double domain[4];
} dc_scene_opts;

/* How one evaluation of the representation is carried out.
 * method: DC_METHOD_FMM or DC_METHOD_DIRECT; precision: DC_PREC_*;
 * p: expansion order (coefficients 0..p, 1 <= p <= DC_P_MAX);
 * tile_px: render target boxes hold at most tile_px x tile_px pixels
 * (2..16); near_fp64: in DC_PREC_F32, a pixel closer to a chord than
 * near_fp64 * (chord length) is evaluated in FP64. */
typedef struct {
    int method;
    int precision;
    int p;
    int tile_px;
    double near_fp64;
} dc_eval_opts;

/* GMRES (Sec. 6.5.1): relative residual tolerance ||b - Ax|| / ||b|| per
 * channel, at most max_iter Arnoldi steps (no restart), initial guess 1.
 * precond = DC_PRECOND_BLOCK applies GMRES to A M^-1 with M the block
 * diagonal of A over the curves (each curve's own hybrid matrix, inverted
 * on the device); the system and its solution are unchanged. */
#define DC_PRECOND_NONE 0
#define DC_PRECOND_BLOCK 1
typedef struct {
    double tol;
    int max_iter;
    dc_eval_opts matvec;
    int precond;
} dc_solve_opts;

typedef struct {
    double cx, cy, width, height;
    int W, H;
} dc_viewport;

typedef struct {
    int iters[3];                  /* Arnoldi steps per channel */
    double rel_residual[3];        /* GMRES estimate at exit */
    double true_rel_residual[3];   /* ||b - A x|| / ||b|| recomputed */
    double seconds;                /* wall time of the solve */
    int converged;                 /* 1 if every channel met tol */
} dc_solve_report;

typedef struct {
    int n_curves, N, S;            /* curves, GL nodes, chord segments */
    int n_pieces;                  /* chords clipped at quadtree leaves */
    int n_cells, n_leaves, depth;  /* quadtree size */
    double root[3];                /* root box x0, y0, side */
    int solved;                    /* densities present */
    long long table_pairs;         /* (node, piece) pairs in the solve's
                                      near-field tables (0: none built) */
    long long table_bytes;         /* device bytes they hold */
} dc_scene_info;

/* Fill opts / eval with the library defaults (P=16, g=16, s=80, b=64,
 * max_depth=40, domain [-0.45,1.45]^2; FMM, FP64, p=20, tile 8, near 1e-3). */
void dc_default_scene_opts(dc_scene_opts* opts);
void dc_default_eval_opts(dc_eval_opts* eval);

/* Build a scene: arc-length parametrisation (App. B), panels, GL nodes,
 * chord segments with their arc-length scale (App. A), boundary values
 * from the colour stops, the quadtree over the nodes and the chords
 * clipped at its leaves (Sec. 6.1, 6.2), all copied to the device.
 * Synchronous.  DC_ERR_INVALID for NaN/Inf input, a zero-length curve,
 * n_stops < 2 or bad options. */
int dc_scene_create(const double* ctrl, int n_curves,
                    const double* left_rgb, const double* right_rgb,
                    int n_stops, const dc_scene_opts* opts, dc_scene* out);

void dc_scene_destroy(dc_scene s);

int dc_scene_get_info(dc_scene s, dc_scene_info* info);

/* Node positions, host [N][2], in node order.  Synchronous. */
int dc_get_nodes(dc_scene s, double* xy_host);

/* Replace the boundary values with arbitrary nodal data, host [3][N] each
 * (u+ on the left side, u- on the right).  Drops solved densities. */
int dc_set_boundary(dc_scene s, const double* u_plus_host,
                    const double* u_minus_host);

/* Alg. 3: mu = u+ - u-, b = (u+ + u-)/2 - F_H mu, sigma = GMRES(G_H, 1, b).
 * Densities stay resident on the device.  Synchronous (returns after the
 * solve).  DC_ERR_NOT_CONVERGED keeps the last iterate as the densities. */
int dc_solve_densities(dc_scene s, const dc_solve_opts* o,
                       dc_solve_report* rep, void* stream);

/* Sec. 5.4 (mixed conditions, Eq. neumann_mat): one-sided Dirichlet and
 * Neumann data on closed curves, for the domain the curves enclose on their
 * left (counter-clockwise loops: the left normal points into it).  At every
 * node 1/2 u = G_H psi + F_H u, with psi the normal derivative of u along
 * the outward normal (right normal).  neumann (host [N], 0 or 1) marks the
 * Neumann nodes; values (host [3][N]) holds u* at Dirichlet nodes and psi*
 * at Neumann nodes.  GMRES (Sec. 6.5.1; o->precond must be
 * DC_PRECOND_NONE) solves for psi on the Dirichlet nodes and u on the
 * Neumann nodes; the scene then holds sigma = psi and mu = u, so dc_render
 * evaluates u(x) = int G psi + F u inside (the scene's two-sided colour data
 * come back with the next dc_solve_densities, dc_set_densities or
 * dc_set_boundary).  Every curve of the scene must belong to such a loop.
 * Synchronous; errors as dc_solve_densities. */
int dc_solve_mixed(dc_scene s, const int* neumann, const double* values,
                   const dc_solve_opts* o, dc_solve_report* rep, void* stream);

/* ---------------------------------------------------------------------
 * Adaptive subdivision with local re-solve (Sec. 7: Alg. 5, 6, 7).
 *
 * A panel is the piece of curve c between normalised arc lengths lo < hi;
 * it carries g GL nodes and s chord segments like the equal panels of
 * dc_scene_create.
 *
 * dc_scene_create_panels: a scene from an explicit panel list (host arrays
 * [n_panels]: panel_curve, panel_lo, panel_hi; panels listed curve by
 * curve, in order along each, not overlapping); opts->panels_per_curve is
 * ignored.  Otherwise as dc_scene_create.
 *
 * dc_scene_panels: the scene's panel count, and its panel list when the
 * arrays (host, [n_panels] each) are not null.  Synchronous.
 *
 * dc_panel_tails: tails[k] (host [n_panels]) = max over the colour channels
 * of |a_{g-1}|, the highest coefficient of the Legendre expansion of the
 * density on panel k, a_k = (2k+1)/2 sum_i w_i sigma_i P_k(x_i) (Alg. 5's
 * test).  Needs densities.  Synchronous.
 *
 * dc_refine: rounds of Alg. 7 on a solved scene made from colour stops
 * (not after dc_set_boundary or dc_solve_mixed).  Each round cuts every
 * panel whose tail exceeds eps2, whose arc length is at least eps1 and one
 * of whose chords meets the viewport (viewport[2] <= 0: anywhere) at its
 * arc-length midpoint (Alg. 5); builds the new scene (same options and
 * colour stops); starts from the old densities interpolated to the new
 * nodes (Sec. 7.1.1); with local = 1 labels the re-solving curves --
 * the cut curves and every curve S_b with max - min of G_H rho over S_b
 * above ratio times that over S_a, rho = 1 on a cut curve S_a (Sec.
 * 7.1.4) -- and solves only for their densities, the other curves' held
 * (Eq. local_resolve_mat, with b = (u+ + u-)/2 - F_H mu computed at the new
 * nodes); local = 0 re-solves every curve.  Rounds stop when no panel is
 * cut or after max_rounds.  *out receives the refined scene (the caller
 * destroys it), or NULL when the first round cut nothing; s is unchanged.
 * resolved (host [n_curves], may be NULL) receives the last round's labels
 * (1 = re-solved).  Synchronous.  DC_ERR_NOT_CONVERGED when a re-solve
 * missed the tolerance (*out is still set). */
typedef struct {
    double eps2;          /* Legendre tail threshold (density units) */
    double eps1;          /* shortest panel that may be cut (arc length) */
    double viewport[4];   /* cx, cy, width, height of the region to refine */
    double ratio;         /* re-solving rule of label_curves (0.9) */
    int max_rounds;       /* rounds of Alg. 7 at most */
    int local;            /* 1: local re-solve (Alg. 6); 0: every curve */
    dc_solve_opts solve;  /* GMRES of the re-solves */
} dc_refine_opts;

typedef struct {
    int rounds;            /* rounds that cut panels */
    int panels_cut;        /* panels cut, all rounds */
    int n_panels;          /* panels of the refined scene */
    int curves_resolved;   /* re-solving curves, summed over the rounds */
    int iters;             /* GMRES steps (largest channel), summed */
    int converged;         /* every re-solve met the tolerance */
    double rel_residual;   /* largest true relative residual of a re-solve */
    double seconds;        /* wall time */
    double label_seconds;  /* of which labelling the re-solving curves */
    double solve_seconds;  /* of which GMRES */
} dc_refine_report;

/* eps2 = 1, eps1 = 0, whole scene, ratio 0.9, one round, local; the solve
 * options: tol 1e-10, 500 steps, block preconditioner, FMM FP64 p = 20. */
void dc_default_refine_opts(dc_refine_opts* o);
int dc_scene_create_panels(const double* ctrl, int n_curves,
                           const double* left_rgb, const double* right_rgb,
                           int n_stops, const int* panel_curve,
                           const double* panel_lo, const double* panel_hi,
                           int n_panels, const dc_scene_opts* opts,
                           dc_scene* out);
int dc_scene_panels(dc_scene s, int* n_panels, int* panel_curve,
                    double* panel_lo, double* panel_hi);
int dc_panel_tails(dc_scene s, double* tails_host, void* stream);
int dc_refine(dc_scene s, const dc_refine_opts* o, dc_scene* out,
              dc_refine_report* rep, unsigned char* resolved_host,
              void* stream);

/* Cached near-field tables of the solve (Sec. 6.4, the precomputed
 * operators reused by every GMRES matvec).  The near field of the FP64
 * operator depends on the geometry alone: on the first FP64 FMM operator
 * application (dc_solve_densities, dc_apply_operator, ...) the library
 * can store each target leaf's near pieces and separated boxes and the
 * chord integrals of every (node, near piece) pair, so that later
 * applications read them instead of walking the tree and evaluating the
 * closed forms (same values; sums in another order).  mode = 1 (the
 * default): built when they fit 16 GiB and the near field averages at
 * least 256 pairs per node (large leaf capacities; sparser near fields
 * evaluate as fast as the tables read); mode = 2: whenever they fit;
 * mode = 0: never (as the FP32 operator).  Mode 2 also keeps, for every
 * operator application (FP64 or FP32), the density-free factors of each
 * piece's outgoing expansion (n_pieces x (p + 1) x 32 bytes, at most
 * 8 GiB) and reads them instead of recomputing them: the same values.
 * Every call drops the tables built so far.  dc_scene_get_info reports the
 * near-field tables' size.  Synchronous. */
int dc_set_solve_tables(dc_scene s, int mode);

/* Densities sigma at the nodes, host [3][N].  Synchronous. */
int dc_get_densities(dc_scene s, double* sigma_host);

/* Install densities (e.g. from a checkpoint), host [3][N].  Synchronous. */
int dc_set_densities(dc_scene s, const double* sigma_host);

/* y = G_H x + c_mu * F_H mu at the nodes (the solve's operator, Eq.
 * db_mat_solve), x_dev and y_dev device [3][N] FP64 in node order.
 * c_mu is 0 or 1.  Asynchronous on stream. */
int dc_apply_operator(dc_scene s, const double* x_dev, double* y_dev,
                      int c_mu, const dc_eval_opts* o, void* stream);

/* Alg. 4: u = FMM_G(Pi sigma) + FMM_F(Pi mu) at every pixel centre of vp,
 * written to out_dev ([H][W][3], FP32 or FP64 per out_dtype).  Needs
 * densities.  Every pixel centre must lie inside the quadtree root.
 * Asynchronous on stream.  Renders of one scene share its device scratch:
 * when they are issued on different streams the caller orders them (the
 * server below has scratch of its own).  A large render (8-pixel tiles,
 * at least 65,536 of them) runs part of its pixel pass on a second stream
 * of the scene; that work is joined back into stream by an event before
 * the call returns, so stream alone orders the result.  That second stream
 * and its two events are used under a lock of the scene, so a direct render
 * of a scene registered with a server may be issued from another host
 * thread while the server's worker renders the same scene. */
int dc_render(dc_scene s, const dc_viewport* vp, const dc_eval_opts* o,
              int out_dtype, void* out_dev, void* stream);

/* dc_render for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, images and error codes as dc_render (o->method must be
 * DC_METHOD_FMM); the image is bit-identical to dc_render's.  It calls no
 * hipMalloc, hipFree, pinned-host allocation or stream creation: the render's
 * device scratch is a fixed array of DC_NOALLOC_SCRATCH_BYTES bytes that
 * each GPU the library runs on holds until the process ends, the render's
 * descriptor tables reach it as kernel arguments, and every launch goes on
 * stream (no second stream).  Requirements, each refused with
 * DC_ERR_INVALID: the scene must already be prepared for o's order and
 * precision (an earlier dc_render, dc_render_batch or dc_server_add_scene
 * with the same p and precision made its resident expansions), and the
 * render's scratch must fit the array (roughly 34 bytes per pixel with
 * 8-pixel tiles and 4 with 16-pixel tiles at p = 12).  All calls on one GPU
 * share that GPU's array and the array keeps the last call's contents:
 * calls that overlap on one GPU (on different streams without ordering
 * between them) race; calls on one stream are ordered. */
#define DC_NOALLOC_SCRATCH_BYTES (64LL << 20)
int dc_render_noalloc(dc_scene s, const dc_viewport* vp, const dc_eval_opts* o,
                      int out_dtype, void* out_dev, void* stream);

/* Alg. 4 for n viewports of one scene in one set of launches: one
 * downward launch per quadtree level covers every viewport that reaches
 * that level and one leaf pass covers every viewport's pixel tiles (the
 * viewports are independent, so this is a batching of Alg. 4, not a change
 * of what it computes).  vps[v] and outs[v] (device [H][W][3], FP32 or FP64
 * per out_dtype) as in dc_render; each image equals dc_render of its
 * viewport alone.  o->method must be DC_METHOD_FMM.  n >= 1; the host
 * arrays are read before the call returns.  Asynchronous on stream; the
 * descriptor tables are copied from host memory owned by the scene, so a
 * second batch call on the same scene waits for nothing but must not run
 * concurrently on another stream. */
int dc_render_batch(dc_scene s, const dc_viewport* vps, int n,
                    const dc_eval_opts* o, int out_dtype, void* const* outs_dev,
                    void* stream);

/* Sec. 8 (anti-aliasing): the render of dc_render in which every pixel whose
 * closed square meets a chord segment of the scene takes the mean of the
 * representation at the centres of its aa x aa equal sub-squares (an
 * area-weighted sum over one level of sub-cells, the paper's recursive
 * area weighting near curves); every other pixel keeps its centre value.
 * Pixel (r, k) covers [x0 + k pw, x0 + (k+1) pw] x [y1 - (r+1) ph, y1 - r ph]
 * with x0 = cx - width/2, y1 = cy + height/2, pw = width/W, ph = height/H;
 * its sub-square (i, j) is centred at (x0 + (k + (i + 1/2)/aa) pw,
 * y1 - (r + (j + 1/2)/aa) ph).  The sub-square samples are rendered by the
 * FMM with o (method FMM) as small viewports in one batched render, so
 * unlike the paper's scheme the image size need not be a power of two.
 * aa in 2..16.  rep (may be NULL) receives the number of anti-aliased
 * pixels, of pixel blocks rendered at aa x aa samples and of samples.
 * Synchronous (returns after out_dev is written); other arguments, errors
 * and ownership as in dc_render. */
typedef struct {
    long long aa_pixels;   /* pixels replaced by sub-square means */
    int blocks;            /* batched sub-viewports (blocks of edge pixels) */
    long long samples;     /* sub-square samples rendered */
} dc_aa_report;
int dc_render_aa(dc_scene s, const dc_viewport* vp, const dc_eval_opts* o, int aa,
                 int out_dtype, void* out_dev, dc_aa_report* rep, void* stream);

/* Render options chosen on the device against an accuracy target.  For each
 * tile size in tiles[0..n_tiles), orders p = p_min, p_min + p_step, ... up to
 * p_max are tried in turn on the viewports vps[0..n) (one batched render per
 * order) until the largest |FMM - direct| over the sampled pixels is at most
 * target_err; the reference is the FP64 direct sum over every chord segment
 * at those pixel centres (the representation of Alg. 4 without the FMM, on
 * the scene's own geometry), so no external values are needed.  About
 * `samples` pixels per viewport are checked: half on a stride grid and half
 * along the chords that cross the viewport (the near field).  The chosen
 * order of each tile size is then timed over timing_reps renders, and the
 * fastest tile size that met the target is returned in rep->chosen (if none
 * met it, the most accurate one, with rep->met = 0).  The leaf capacity is a
 * property of the scene (dc_scene_opts) and is not tuned here.  The scene
 * must have densities and must not be registered with a server; it is left
 * prepared for the chosen options (dc_render_noalloc may follow).
 * Synchronous.  DC_ERR_INVALID for bad options (n_tiles in 1..4, tiles in
 * 2..16, 1 <= p_min <= p_max <= DC_P_MAX, p_step >= 1, samples >= 2,
 * timing_reps >= 1, target_err > 0). */
typedef struct {
    double target_err;
    int precision;               /* DC_PREC_F32 or DC_PREC_F64 */
    int p_min, p_max, p_step;
    int tiles[4];
    int n_tiles;
    int samples;                 /* sampled pixels per viewport */
    double near_fp64;            /* as in dc_eval_opts */
    int timing_reps;
} dc_tune_opts;

typedef struct {
    dc_eval_opts chosen;         /* method FMM, the tuned p and tile_px */
    double err;                  /* max |FMM - direct| at the samples, chosen */
    double ms;                   /* ms per render of all viewports, chosen */
    int n_samples;               /* sampled pixels over all viewports */
    int met;                     /* 1 when err <= target_err */
    int tile_p[4];               /* per tile size tried: the order reached */
    double tile_err[4];          /* its error */
    double tile_ms[4];           /* its time (ms per render of all viewports) */
} dc_tune_report;

/* Defaults: target 5e-5 (half the 1e-4 bar of the FP32 path), FP32,
 * p = 8, 10, ..., 24, tiles {8, 16}, 1024 samples per viewport, near 1e-3,
 * 5 timing renders. */
void dc_default_tune_opts(dc_tune_opts* t);
int dc_autotune(dc_scene s, const dc_viewport* vps, int n, const dc_tune_opts* t,
                dc_tune_report* rep, void* stream);

/* The same representation at n arbitrary points xy_dev (device [n][2]
 * FP64), out_dev [n][3].  Uses the direct sum (method is ignored). */
int dc_eval_points(dc_scene s, const double* xy_dev, int n,
                   const dc_eval_opts* o, int out_dtype, void* out_dev,
                   void* stream);

/* Work actually done by one render, counted on the device (the counting
 * run is separate from timed runs).  Synchronous. */
typedef struct {
    unsigned long long p2p_pairs;       /* (target, piece) closed forms */
    unsigned long long p2p_fp64_pairs;  /* of those, evaluated in FP64 */
    unsigned long long m2p_pairs;       /* (target, box) outgoing evaluations */
    unsigned long long l2p_targets;     /* targets evaluated from an incoming expansion */
    unsigned long long m2l_pairs;       /* (target box, source box) translations */
    unsigned long long p2l_pairs;       /* (target box, piece) incoming-from-source */
    unsigned long long p2l_fp64_pairs;  /* of those, evaluated in FP64 */
    unsigned long long l2l_boxes;       /* parent-to-child incoming translations */
    unsigned long long leaf_boxes;      /* target leaves evaluated */
    unsigned long long pieces;          /* clipped chord pieces of the scene */
    unsigned long long source_cells;    /* boxes of the source quadtree */
    int levels;                         /* levels of the target tree */
    int p;                              /* expansion order used */
} dc_work_counts;

int dc_render_counts(dc_scene s, const dc_viewport* vp, const dc_eval_opts* o,
                     dc_work_counts* counts, void* stream);

/* Repeated renders without per-call launch work: the launches of one
 * dc_render_batch (same arguments; FMM only) captured into a HIP graph that
 * dc_render_graph_launch replays on a stream, for callers that render the
 * same viewports into the same output buffers again and again (frames of
 * an unchanged view, benchmarks).  The graph owns its plan, descriptor
 * tables and device scratch, so it does not share scratch with dc_render;
 * outs[v] must stay allocated while the graph exists.  The scene's
 * densities must be set; the upward pass for o's order and precision is
 * done (and waited for) during the call.  Launch fails with
 * DC_ERR_INVALID when the densities changed since the capture, or when the
 * resident expansions were rebuilt for another order or precision (a
 * render with other options; their buffers may have moved): make the
 * graph again.  Not for a scene registered with a server.  Destroy waits
 * for the device. */
typedef struct dc_render_graph_s* dc_render_graph;
int dc_render_graph_create(dc_scene s, const dc_viewport* vps, int n,
                           const dc_eval_opts* o, int out_dtype,
                           void* const* outs_dev, dc_render_graph* out);
int dc_render_graph_launch(dc_render_graph g, void* stream);
void dc_render_graph_destroy(dc_render_graph g);

/* Per-phase timing of dc_render with HIP events on the caller's stream.
 * While enabled every dc_render waits for its own completion.
 * dc_get_timing fills ms[5] = {upward, downward, leaf, total (ms, summed
 * over calls), number of calls} and resets the sums. */
int dc_set_timing(dc_scene s, int enable);
int dc_get_timing(dc_scene s, double* ms);

/* ------------------------------------------------------------------------
 * Serving: a render loop over resident scenes with continuous batching.
 *
 * Alg. 4 is evaluated once per request (a viewport of a registered scene)
 * exactly as dc_render does, so a result does not depend on which other
 * requests share its batch.  A worker thread owned by the server takes
 * queued requests in arrival order, groups the oldest request with later
 * requests of the same scene (up to max_batch requests and
 * max_batch_pixels pixels), and admits the group when its device footprint
 * (images plus render scratch, computed exactly from the render plan) fits
 * in the free part of an arena of hbm_budget bytes; otherwise the oldest
 * request waits (no reordering past it) until completed batches or fetched
 * images free memory.  Admitted batches run on up to n_streams HIP streams
 * at once, so batches of different scenes and new arrivals overlap on the
 * device with batches already running.  Images stay in the arena until
 * fetched: a client that never fetches eventually blocks admission.
 *
 * Threading: submit, wait, fetch and get_stats may be called from any host
 * threads.  A registered scene is read-only: dc_solve_densities,
 * dc_set_densities, dc_set_boundary and dc_apply_operator fail on it, renders
 * must use the order and precision it was registered with, and
 * dc_scene_destroy leaves it alive, until dc_server_destroy.
 * ------------------------------------------------------------------------ */
typedef struct dc_server_s* dc_server;

typedef struct {
    dc_eval_opts eval;          /* options of every render (method FMM) */
    int out_dtype;              /* DC_OUT_F32 or DC_OUT_F64 */
    int n_streams;              /* batches in flight at once, 1..16 */
    int max_batch;              /* requests per batch, >= 1 */
    long long max_batch_pixels; /* pixels per batch, >= 1 */
    long long hbm_budget;       /* device bytes for images + scratch */
} dc_server_opts;

typedef struct {
    double t_submit, t_start, t_done;  /* seconds since server creation:
                                          submitted, launched, observed done */
    long long batch;                   /* id of the batch that rendered it */
    int batch_size;                    /* requests in that batch */
    int status;                        /* DC_OK or the batch's error code */
    long long bytes;                   /* image bytes held until fetched */
} dc_request_info;

typedef struct {
    long long submitted, completed, fetched, batches;
    long long max_in_flight;           /* most batches running at once */
    long long bytes_in_use, bytes_peak;
    long long admission_waits;         /* admissions deferred for memory */
} dc_server_stats;

/* Defaults: FMM FP32 p=12 tile 8, FP32 images, 4 streams, 64 requests and
 * 2^26 pixels per batch, 8 GiB. */
void dc_default_server_opts(dc_server_opts* o);

/* Create a server on the current HIP device: allocates the arena (one
 * hipMalloc of hbm_budget bytes), the streams and the worker thread. */
int dc_server_create(const dc_server_opts* o, dc_server* out);

/* Register a scene with densities and run its upward pass for the server's
 * options (synchronous).  The scene must live on the server's device. */
int dc_server_add_scene(dc_server sv, dc_scene s);

/* The same with render options of the scene's own (method FMM; e.g. the
 * order and tile size dc_autotune chose for it): every request of the scene
 * is rendered with *o, requests of other scenes with theirs.  Images are
 * written in the server's out_dtype.  Registering a scene again with other
 * options fails with DC_ERR_INVALID. */
int dc_server_add_scene_opts(dc_server sv, dc_scene s, const dc_eval_opts* o);

/* Queue a render of vp of registered scene s; *ticket identifies it.
 * Fails with DC_ERR_INVALID for a viewport outside the scene's quadtree
 * root and DC_ERR_OOM when the request alone exceeds hbm_budget. */
int dc_server_submit(dc_server sv, dc_scene s, const dc_viewport* vp,
                     long long* ticket);

/* Wait up to timeout_s seconds (< 0: no limit) for a request; fills info
 * (may be NULL).  DC_OK when it is done, DC_ERR_TIMEOUT otherwise. */
int dc_server_wait(dc_server sv, long long ticket, double timeout_s,
                   dc_request_info* info);

/* Copy a finished request's image ([H][W][3] of out_dtype) to dst (device
 * memory when dst_is_device, else host) and release it; the ticket is then
 * forgotten.  Synchronous. */
int dc_server_fetch(dc_server sv, long long ticket, void* dst, int dst_is_device);

int dc_server_get_stats(dc_server sv, dc_server_stats* st);

/* Finish every queued and running request, then free the server (unfetched
 * images are dropped) and unregister its scenes. */
void dc_server_destroy(dc_server sv);

const char* dc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DCFMM_H */
