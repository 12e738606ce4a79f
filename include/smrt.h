/*
 * smrt.h -- C ABI of the MI355X (gfx950) D2Q9 lattice Boltzmann library for
 * the single MRT-featured collision (SmrtLBM) and the single-relaxation-time
 * (SRT/BGK) collision of Zhou, "Single MRT-featured Lattice Boltzmann Method"
 * (arXiv:2409.01076).
 *
 * What one step computes (lattice units, dx = dt = e = 1):
 *   streaming   f_a(x, t+1) = f*_a(x - e_a, t), the left-hand side of
 *               Eq. (lb.srt) / Eq. (SmrtLBM-1) written in pull form;
 *   moments     rho = sum_a f_a, u = sum_a e_a f_a / rho           (Eq. fea-0);
 *   equilibrium f^eq_a(rho, u)                                     (Eq. feq-full);
 *   collision   SRT     f* = f - (f - f^eq)/tau                    (Eq. lb.srt)
 *               SmrtLBM f*_a = f^eq_a + (-1)^a (1 - 1/tau) C_g(a)  (Eq. SmrtLBM-1,
 *                       with the group sums C_1, C_2 of Eq. sigma1-2-0)
 *               TRT     f*_a = f_a - (f_a - f^eq_a)/tau_s
 *                              + (-1)^a (1/tau_s - 1/tau) C_g(a)   (Eq. SmrtLBM-lb.1.5)
 *   walls       cavity: the "standard bounce-back" of the cavity section, read as
 *               half-way bounce-back (walls half a link outside the outer nodes);
 *               the top wall moves at (u_lid, 0) and adds 6 w_a (e_a . u_w) to the
 *               bounced population (moving-wall bounce-back, wall density 1); links
 *               that end in the row above the top nodes, corners included, end on
 *               the lid.  periodic: both axes wrap.
 *
 * Layout: the library stores the post-collision populations as deviations
 * d_a = f*_a - w_a in structure-of-arrays planes (one plane per direction,
 * rows of nx nodes, x fastest, y = 0 the bottom row) inside a device workspace.
 * Every array passed in or out below is a dense device array: fields are
 * [ny][nx], populations are [9][ny][nx] full values f (not deviations).
 *
 * Threads and streams: a context is used by one host thread at a time.  All
 * device work is enqueued on the stream given at creation (NULL = the default
 * stream); calls return without waiting unless stated.
 *
 * Errors: every int-returning call returns SMRT_OK (0) or a negative
 * smrt_status; smrt_last_error() then gives a message for the calling thread.
 * No C++ exception crosses this interface.
 */
#ifndef SMRT_H
#define SMRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum smrt_status {
    SMRT_OK = 0,
    SMRT_EINVAL = -1,    /* invalid argument (size, enum, relaxation time, pointer) */
    SMRT_ENOMEM = -2,    /* workspace too small or allocation failed               */
    SMRT_EDEVICE = -3,   /* a HIP runtime call or kernel launch failed             */
    SMRT_EUNSTABLE = -4, /* the state holds a non-finite density or velocity       */
    SMRT_ESTATE = -5     /* call not valid in the current state                    */
} smrt_status;

typedef enum smrt_scheme {
    SMRT_SCHEME_SRT = 0,  /* Eq. (lb.srt)          */
    SMRT_SCHEME_SMRT = 1, /* Eq. (SmrtLBM-1)       */
    SMRT_SCHEME_TRT = 2   /* Eq. (SmrtLBM-lb.1.5)  */
} smrt_scheme;

typedef enum smrt_boundary {
    SMRT_CAVITY = 0,      /* lid-driven square cavity of the paper's test section */
    SMRT_PERIODIC = 1,    /* both axes wrap around                                */
    SMRT_CAVITY_EQLID = 2 /* the cavity under a second reading of its lid: the top
                             row of nodes is the lid, set each step to
                             f^eq(rho, (u_lid, 0)) (Eq. feq-full) with
                             rho - 1 = d_0 + d_1 + d_3 + 2 (d_2 + d_5 + d_6) from the
                             populations it received; side and bottom walls
                             half-way bounce-back.  One time step per launch. */
} smrt_boundary;

typedef enum smrt_dtype {
    SMRT_F64 = 0,
    SMRT_F32 = 1,
    SMRT_F16 = 2, /* storage only: IEEE binary16 deviations, FP32 arithmetic */
    SMRT_BF16 = 3,/* storage only: bfloat16 deviations, FP32 arithmetic      */
    SMRT_F32X = 4,/* storage only: binary32 deviations, FP64 arithmetic: each
                     collision is computed in FP64 and rounded once per stored
                     value, so the only FP32 error is the storage's own
                     (about 5x below SMRT_F32's on a slowly converging
                     cavity; SMRT_F32 takes 1/12 of the diagonal links' odd
                     equilibrium terms as a pair of binary32 constants, since
                     one rounded constant biases every node alike) */
    /* Moment storage (SmrtLBM only; cavity or periodic; one time step per
     * launch).  Eq. (SmrtLBM-1) makes the post-collision populations a
     * function of five numbers per node, f*_a = f^eq_a(rho, u) + (-1)^a g_grp(a)
     * with g_1 = (1 - 1/tau) C_1 (axis links) and g_2 = (1 - 1/tau) C_2
     * (diagonal links), so the state is stored as rho - 1, j = rho u and g_1,
     * g_2, and each step rebuilds the pulled populations from the
     * neighbours' moments.  The large equilibrium part keeps binary32 (or
     * FP64) precision and the small amplitudes, which carry the viscous
     * stress, get their own 16-bit relative precision. */
    SMRT_M64 = 5,  /* FP64 moments and amplitudes, FP64 arithmetic (40 B a node) */
    SMRT_M16 = 6,  /* binary32 moments, FP16 amplitudes (scaled by 2^12), FP32
                      arithmetic: 16 B a node */
    SMRT_MBF16 = 7 /* binary32 moments, bfloat16 amplitudes, FP32 arithmetic:
                      16 B a node */
} smrt_dtype;

typedef struct smrt_params {
    int32_t nx, ny;    /* lattice nodes along x and y, each >= 3             */
    int32_t scheme;    /* smrt_scheme                                        */
    int32_t boundary;  /* smrt_boundary                                      */
    int32_t storage;   /* smrt_dtype of the stored state; arithmetic is FP64
                          for SMRT_F64, SMRT_F32X and SMRT_M64, FP32
                          otherwise                                          */
    int32_t reserved0; /* must be 0                                          */
    double tau;        /* > 1/2: used as given.  <= 0: derived from re as
                          tau = 3 |u_lid| nx / re + 1/2, i.e.
                          Eq. (relation-chapman-viscosity) with
                          nu = |u_lid| nx / re                               */
    double re;         /* Reynolds number, used only when tau <= 0           */
    double u_lid;      /* lid speed (cavity), |u_lid| < 1/sqrt(3)            */
    double tau_s;      /* TRT only: relaxation time of the other moments, > 1/2 */
    void* stream;      /* hipStream_t, NULL for the default stream           */
    int64_t reserved[4]; /* must be 0                                        */
} smrt_params;

typedef struct smrt_ctx smrt_ctx;

/* Device workspace bytes needed by a context with these parameters (two
 * population buffers, the residual snapshot and reduction scratch); 0 if the
 * parameters are invalid.  Pure host computation. */
size_t smrt_workspace_bytes(const smrt_params* p);

/* Creates a context and sets the cold start f = f^eq(rho = 1, u = 0), t = 0.
 * dev_ws: caller-owned device memory of at least smrt_workspace_bytes(p)
 * bytes, 256-byte aligned, kept alive until smrt_destroy; or NULL to let the
 * library allocate (and later free) it.  ws_bytes is ignored when dev_ws is
 * NULL.  SMRT_EINVAL: nx or ny < 3, nx * ny > 2^34, a row of more than
 * 2 MiB of stored values (nx > 262,144 for SMRT_F64, 524,288 for SMRT_F32,
 * 1,048,576 for 16-bit storage: the kernels address a tile through 32-bit
 * byte offsets), unknown enum, moment storage with a scheme other than
 * SmrtLBM or with SMRT_CAVITY_EQLID, relaxation time <= 1/2, |u_lid| >= 1/sqrt(3),
 * non-zero reserved fields, out == NULL.  SMRT_ENOMEM:
 * ws_bytes too small or the allocation failed.  On error *out is NULL. */
int smrt_create(const smrt_params* p, void* dev_ws, size_t ws_bytes, smrt_ctx** out);

/* Sets f = f^eq(rho, u) at every node from dense device fields [ny][nx] of
 * dtype SMRT_F32 or SMRT_F64 (Eq. feq-full); rho == NULL means 1 everywhere,
 * ux/uy == NULL mean 0.  Resets the step counter and the residual snapshot. */
int smrt_init_fields(smrt_ctx* c, const void* rho, const void* ux, const void* uy,
                     int32_t dtype);

/* Replaces the state by the post-collision populations f (device,
 * [9][ny][nx], SMRT_F32 or SMRT_F64, full values), e.g. to resume a run;
 * resets the step counter and the residual snapshot.  Values are rounded to
 * the storage type; moment storage keeps the density, momentum and the two
 * group sums of f - f^eq (Eq. sigma1-2-0) as g_1, g_2, which is exact for any
 * SmrtLBM post-collision state. */
int smrt_set_populations(smrt_ctx* c, const void* f, int32_t dtype);

/* Writes the current post-collision populations f = w + d (device,
 * [9][ny][nx], SMRT_F32 or SMRT_F64). */
int smrt_get_populations(smrt_ctx* c, void* f, int32_t dtype);

/* Enqueues n time steps (streaming, walls, moments, equilibrium, collision,
 * store).  n == 0 does nothing; n < 0 is SMRT_EINVAL.  Asynchronous. */
int smrt_step(smrt_ctx* c, int64_t n);

/* Writes rho, ux, uy of the current state (Eq. fea-0) into dense device
 * arrays [ny][nx] of dtype SMRT_F32 or SMRT_F64; any pointer may be NULL to
 * skip that field.  The moments of the stored post-collision populations equal
 * those of the pre-collision ones because the collision conserves density and
 * momentum.  Asynchronous. */
int smrt_moments(smrt_ctx* c, void* rho, void* ux, void* uy, int32_t dtype);

/* Steady-state residual over the window since the last snapshot:
 *   R = ||u(t) - u(t_snap)||_2 / ((t - t_snap) ||u(t)||_2),
 * summed in FP64 in a fixed order; then u(t) becomes the new snapshot.
 * Synchronizes the stream.  SMRT_ESTATE if no step ran since the snapshot;
 * SMRT_EUNSTABLE (and *out = NaN) if any density or velocity is not finite.
 * R is 0 for a lattice at rest that did not move. */
int smrt_residual(smrt_ctx* c, double* out);

/* Total mass sum rho in FP64, fixed summation order.  Synchronizes the
 * stream.  SMRT_EUNSTABLE (and *out = NaN) on a non-finite value. */
int smrt_mass(smrt_ctx* c, double* out);

/* For callers that cannot allocate or synchronize: code under HIP graph
 * capture, serving loops that forbid allocation, harnesses without hipMalloc.
 * The mass of smrt_mass, enqueued on the context's stream without a host
 * round trip: dev_out (device, 2 doubles) receives sum rho in FP64 (the same
 * kernels and fixed summation order as smrt_mass, so the same value) and the
 * number of nodes holding a non-finite density or velocity (0 when stable).
 * Allocates nothing: the partial sums live in a static device array of the
 * library, 2048 x 4 + 4 doubles (65.6 KB) on each GPU it runs on, kept until
 * the process ends; its address on a device is taken when the first context
 * is created on that device.  Every partial is rewritten by each call, so no
 * clearing is needed; calls that overlap on one GPU (several streams or
 * host threads) share the array and race.  Asynchronous.  SMRT_EINVAL for
 * NULL arguments or a reduction wider than the static array (never for
 * lattices the library accepts); SMRT_EDEVICE if a launch fails. */
int smrt_mass_noalloc(smrt_ctx* c, double* dev_out);

/* Steps taken since creation or the last state reset. */
int64_t smrt_steps_done(const smrt_ctx* c);

/* Relaxation time in use (after the Re mapping); NaN for c == NULL. */
double smrt_tau(const smrt_ctx* c);

/* Threads per block along x and y, and rows per thread, for the
 * stream-collide kernel (tuning; results do not depend on it).  bx * by must
 * be 64, 128, 256, 512 or 1024 and bx a multiple of 16; rows in 1..8.
 * Moment storage: the tile, bx = 64 and by * rows = 8 or 16 (default 8).
 * SMRT_EINVAL otherwise. */
int smrt_set_launch(smrt_ctx* c, int32_t bx, int32_t by, int32_t rows);

/* Time steps per kernel launch: 1 .. 5 (FP64 storage 1 .. 4).  The
 * multi-step kernels keep the intermediate steps on chip: with S steps, step
 * t+1 is held in LDS on the tile plus a ring of S - 1 nodes, each later step
 * on a ring one node narrower, written over the same LDS.  HBM traffic per
 * node-update falls to 1/S.  Tiles (tile_cols x tile_rows): two steps {64 x
 * 4, 64 x 8, 64 x 16, 64 x 32, 128 x 4, 128 x 8} (0 = 64 x 8); three and four
 * steps {64 x 8, 64 x 16, 64 x 24, 64 x 26} (0 = 64 x 16); five steps
 * {64 x 16, 64 x 22} (0 = 64 x 16); FP64 storage (twice the LDS per node) two
 * steps {64 x 4, 64 x 8}, three steps {64 x 8}, four steps {64 x 8, 64 x 10}
 * (0 = 64 x 8).  Four- and five-step tiles of 512 nodes or more and two-step
 * 64 x 32 tiles run 768 threads per workgroup, other tiles of 1024 nodes or
 * more 512, the rest 256.  A periodic lattice needs nx >= tile_cols + 2r and
 * ny >= tile_rows + 2r with r = steps - 1.  Per node the arithmetic is
 * unchanged: results are bitwise those of single-step launches.  Default at
 * creation: FP32 storage 5 steps with a 64 x 22 tile while that gives >= 1024
 * tiles or while 64 x 16 tiles would need between one and two waves of two
 * workgroups per CU, else with 64 x 16 while that gives >= 256 (SMRT_F32X as
 * SMRT_F32); 16-bit storage 4 steps
 * with a 64 x 26 tile while that gives >= 1024 tiles or (as for FP32) avoids
 * a short second wave with its tiles in one wave, else with 64 x 16
 * while that gives >= 256; smaller lattices 4 steps with 64 x 8 tiles;
 * periodic lattices too small for those rings 2 steps with a 64 x 32 tile
 * while that gives >= 512 tiles, else with 64 x 4; FP64 storage 4 steps with
 * 64 x 10 tiles; lattices too small for the rings: 1.  A step count that is
 * not a multiple ends with one shorter launch (64 x 16 tiles, or 64 x 8 after
 * a mode with shorter tiles).  With steps = 1 the tile arguments are ignored.
 * SMRT_EINVAL if not applicable. */
int smrt_set_steps_per_launch(smrt_ctx* c, int32_t steps, int32_t tile_cols, int32_t tile_rows);

/* Time steps per launch in use (1 .. 5); -1 for c == NULL. */
int32_t smrt_get_steps_per_launch(const smrt_ctx* c);

/* Order in which the multi-step kernels' workgroups take their tiles (a
 * performance knob only: every order computes bitwise the same result).
 * panel_cols = 0: row-major.  panel_cols = P > 0: the tile columns are cut
 * into panels of P, each walked top to bottom, and each of the GPU's 8 XCDs
 * takes one contiguous run of that order, so neighbouring tiles share an L2
 * and the halo rows and columns they both read are fetched from memory once.
 * Default at creation: 16, or one panel for lattices of at most 48 tile
 * columns of 64 nodes (FP64 storage: 32).  SMRT_EINVAL for
 * c == NULL or panel_cols < 0. */
int smrt_set_tile_order(smrt_ctx* c, int32_t panel_cols);

/* Waits for all work enqueued on the context's stream. */
int smrt_synchronize(smrt_ctx* c);

/* Frees what the library allocated; never frees a caller's workspace or
 * stream.  NULL is a no-op.  Does not wait for enqueued work: synchronize
 * first if the workspace is about to be reused. */
void smrt_destroy(smrt_ctx* c);

/* Message describing the last error on the calling thread ("" if none). */
const char* smrt_last_error(void);

/* ------------------------------------------------------------------------
 * Batches: many independent lid-driven cavities (each a square or
 * rectangular cavity of the paper's test section, with its own size and
 * relaxation time) advanced together.  One time step of the whole batch is
 * one kernel launch: a fixed grid of workgroups walks a device table of the
 * tiles of the cavities still running.  Steps run in windows replayed from a
 * captured HIP graph; after each window every running cavity's residual is
 * checked and the cavities that reached the tolerance, or hold a non-finite
 * value, leave the table.  Per node, the arithmetic is that of smrt_step, so
 * a cavity's result does not depend on the batch it runs in.
 * ------------------------------------------------------------------------ */

typedef struct smrt_batch_params {
    int32_t count;        /* number of cavities, >= 1                          */
    int32_t scheme;       /* smrt_scheme                                       */
    int32_t storage;      /* smrt_dtype of the stored populations: SMRT_F64,
                             SMRT_F32, SMRT_F16 or SMRT_BF16 (SMRT_F32X is for
                             single lattices only)                             */
    int32_t reserved0;    /* must be 0                                         */
    const int32_t* nx;    /* host array [count], each >= 3                     */
    const int32_t* ny;    /* host array [count], each >= 3                     */
    const double* tau;    /* host array [count]; NULL or entries <= 0: derived
                             from re as for smrt_params                        */
    const double* re;     /* host array [count] or NULL                        */
    double u_lid;         /* lid speed shared by all cavities                  */
    double tau_s;         /* TRT only                                          */
    void* stream;         /* hipStream_t, NULL for the default stream          */
    int64_t reserved[4];  /* must be 0                                         */
} smrt_batch_params;

typedef struct smrt_batch smrt_batch;

typedef enum smrt_batch_status {
    SMRT_RUNNING = 0,  /* still in the table                                   */
    SMRT_STEADY = 1,   /* residual fell below the tolerance                    */
    SMRT_UNSTABLE = 2  /* a density or velocity became non-finite              */
} smrt_batch_status;

/* Device workspace bytes for a batch (0 if the parameters are invalid). */
size_t smrt_batch_workspace_bytes(const smrt_batch_params* p);

/* Creates a batch, every cavity at the cold start (rho = 1, u = 0), all
 * running.  dev_ws as for smrt_create (caller-owned or NULL).  The library
 * also allocates small device tables, a pinned host buffer and one private
 * capture stream (default priority).  Default launch: 64 x 16 tiles with
 * five time steps per launch (FP32 storage) or three (16-bit storage); FP64
 * storage one step with 64 x 4 blocks; one workgroup per tile.  Errors as for
 * smrt_create, per cavity; also SMRT_EINVAL when the tile table would exceed
 * 2^31 - 1 entries. */
int smrt_batch_create(const smrt_batch_params* p, void* dev_ws, size_t ws_bytes, smrt_batch** out);

/* Enqueues n time steps of every running cavity (asynchronous). */
int smrt_batch_step(smrt_batch* b, int64_t n);

/* Runs windows of `window` steps until every cavity is steady, unstable or
 * has run max_steps steps in this call.  After each window the per-cavity
 * residual (definition of smrt_residual, over that window) is compared with
 * tol and finished cavities leave the table.  steps_out (host [count], may be
 * NULL) receives each cavity's total steps when it finished (or so far);
 * status_out (host [count], may be NULL) its smrt_batch_status; residual_out
 * (host [count], may be NULL) its last residual.  Synchronizes. */
int smrt_batch_run(smrt_batch* b, double tol, int64_t window, int64_t max_steps, int64_t* steps_out,
                   int32_t* status_out, double* residual_out);

/* Chooses the tile shape (bx, by), the time steps per launch and the number
 * of resident workgroups of the batch kernel by timing `steps` real steps (an
 * even number >= 2) of each candidate (the one-step shapes, and except for
 * FP64 storage the two-step kernel with 64 x 4, 64 x 8 and 64 x 16 tiles,
 * the three- and four-step kernels with 64 x 8 and 64 x 16 tiles and the
 * five-step kernel with 64 x 16 and 64 x 22 tiles); keeps the fastest.
 * Multi-step kernels take one tile a workgroup, so only the full grid is
 * tried for them.
 * chosen (host [3], may be NULL) receives bx, by and the grid size;
 * smrt_batch_steps_per_launch reports the steps per launch.  The trial steps
 * advance every running cavity. */
int smrt_batch_autotune(smrt_batch* b, int32_t steps, int32_t* chosen);

/* Sets the batch's launch shape by hand: `steps` time steps per launch on
 * tiles of bx x by nodes.  steps = 1: (bx, by) one of the one-step shapes
 * (64 x 4, 128 x 2, 256 x 1, 32 x 8, 64 x 8, 128 x 4, 256 x 2, 512 x 1);
 * steps = 2 .. 5 (not for FP64 storage): bx = 64 and by = 8, 16 or 22, or
 * by = 4 with two steps.  Shorter remainder launches of a step count use the
 * same tiles.  The grid becomes one workgroup per tile.  SMRT_EINVAL for
 * other shapes; results are bitwise the same for every shape. */
int smrt_batch_set_launch(smrt_batch* b, int32_t bx, int32_t by, int32_t steps);

/* Fields of cavity `index` (dense device arrays [ny][nx], F32 or F64; any may
 * be NULL), from its current state. */
int smrt_batch_moments(smrt_batch* b, int32_t index, void* rho, void* ux, void* uy, int32_t dtype);

/* f = f^eq(rho, u) for cavity `index` (device fields as smrt_init_fields,
 * NULL = rest); resets its snapshot.  Only while the cavity is running and
 * before smrt_batch_run. */
int smrt_batch_init_fields(smrt_batch* b, int32_t index, const void* rho, const void* ux,
                           const void* uy, int32_t dtype);

/* Steps taken by the running cavities since creation. */
int64_t smrt_batch_steps_done(const smrt_batch* b);

/* Number of cavities still running. */
int32_t smrt_batch_running(const smrt_batch* b);

/* Time steps per launch in use (1 .. 5); -1 for b == NULL. */
int32_t smrt_batch_steps_per_launch(const smrt_batch* b);

/* Frees what the library allocated (not the caller's workspace). NULL: no-op. */
void smrt_batch_destroy(smrt_batch* b);

/* ------------------------------------------------------------------------
 * Warm-start network: a coordinate network that maps a node position and the
 * Reynolds number to (rho, u, v) of the steady cavity flow, used to set the
 * initial populations f = f^eq(rho, u) (Eq. feq-full) instead of the uniform
 * cold start.  Inputs p = (x, y, s), with x, y the node centre over the side
 * length and s = log(Re/100)/log(100).  Features: [x, y, s, sin(2 pi B p),
 * cos(2 pi B p)] with the caller's fixed frequency matrix B (fourier x 3);
 * then (layers - 1) SiLU layers of `width` and a linear output layer.
 * Arithmetic: bfloat16 operands on the matrix cores with FP32 accumulation;
 * FP32 master weights, biases, pre-activations (recomputed in the backward
 * pass, not stored) and Adam state; bfloat16 activations.  Gradients over
 * the n rows: FP32 sums over blocks of at least 256 rows (at most 256 blocks),
 * then the blocks summed in a fixed order (results do not depend on
 * scheduling).
 *
 * Parameter layout (FP32, dense, what set/get_params and smrt_mlp_gradient
 * use): for each layer l in order, W_l as [in_l][out_l] row-major, then b_l
 * [out_l]; in_0 = 3 + 2 fourier, out_last = outputs.
 * Row counts n of every call: a multiple of 64, at most max_batch.
 * ------------------------------------------------------------------------ */

typedef struct smrt_mlp_params {
    int32_t inputs;     /* must be 3: (x, y, s)                           */
    int32_t fourier;    /* frequencies in B, 0..64                        */
    int32_t width;      /* hidden width, a multiple of 64 up to 1024      */
    int32_t layers;     /* weight layers (hidden + output), 2..16         */
    int32_t outputs;    /* 1..64                                          */
    int32_t max_batch;  /* rows per call, a multiple of 64                */
    void* stream;       /* hipStream_t, NULL for the default stream       */
    int64_t reserved[4];/* must be 0                                      */
} smrt_mlp_params;

typedef struct smrt_mlp smrt_mlp;

/* Number of FP32 parameters in the dense layout (0 if params are invalid). */
size_t smrt_mlp_param_count(const smrt_mlp_params* p);

/* Device workspace bytes (weights, Adam state, activations of max_batch
 * rows, gradient partials). */
size_t smrt_mlp_workspace_bytes(const smrt_mlp_params* p);

/* Creates a network (dev_ws as for smrt_create).  Parameters must be set
 * before use. */
int smrt_mlp_create(const smrt_mlp_params* p, void* dev_ws, size_t ws_bytes, smrt_mlp** out);

/* Loads parameters (device, dense layout) and the frequency matrix B
 * (device, fourier x 3 FP32); resets the Adam state.  Asynchronous. */
int smrt_mlp_set_params(smrt_mlp* m, const float* params, const float* fourier);

/* Writes the FP32 master parameters (device, dense layout).  Asynchronous. */
int smrt_mlp_get_params(smrt_mlp* m, float* params);

/* out[n][outputs] (device FP32) for points[n][3] (device FP32).  Asynchronous. */
int smrt_mlp_forward(smrt_mlp* m, const float* points, int32_t n, float* out);

/* Kernels of the forward pass (also inside smrt_mlp_gradient and
 * smrt_mlp_train_step).  enable != 0 (the default): one launch for every
 * layer where the network fits the matrix cores' LDS-resident form (input
 * features padded to 64 or 128 columns, width 64 or 128, at most 8 layers,
 * transposed bf16 weights of at most 140,288 bytes: the default 5-layer,
 * width-128 network with up to 30 frequencies); enable == 0: one launch per
 * layer.  Both produce bitwise the same activations, outputs and gradients
 * (the squared-error loss is summed in another block order).  Returns
 * SMRT_OK or SMRT_EINVAL for a NULL network. */
int smrt_mlp_set_fused_forward(smrt_mlp* m, int32_t enable);

/* 1 if the forward pass runs as one launch (enabled and the network fits),
 * 0 if it runs layer by layer, SMRT_EINVAL for a NULL network. */
int smrt_mlp_uses_fused_forward(const smrt_mlp* m);

/* Gradient of the mean squared error sum (y - target)^2 / (n outputs) with
 * respect to the parameters, into grad (device, dense layout); target is
 * [n][outputs] (device FP32).  loss (host, may be NULL) receives the error
 * (then the call synchronizes). */
int smrt_mlp_gradient(smrt_mlp* m, const float* points, const float* target, int32_t n, float* grad,
                      double* loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * mean squared error of this batch.  loss as above. */
int smrt_mlp_train_step(smrt_mlp* m, const float* points, const float* target, int32_t n, float lr,
                        double* loss);

/* Frees what the library allocated.  NULL: no-op. */
void smrt_mlp_destroy(smrt_mlp* m);

/* The network's matrix product on the matrix cores, exposed for checks and
 * reuse: for each split s < splits,
 *   C[s][m][n] = sum_{k in split s} opA(m, k) opB(k, n),
 *   opA(m, k) = trans_a ? A[k lda + m] : A[m lda + k],
 *   opB(k, n) = trans_b ? B[n ldb + k] : B[k ldb + n],
 * A, B bfloat16 bit patterns (device, 16-byte aligned), C FP32 (device,
 * splits blocks of M x ldc).  M and N multiples of 64, K a multiple of
 * 32 * splits, lda and ldb multiples of 8; split s covers k in
 * [s K/splits, (s+1) K/splits).  SMRT_EINVAL otherwise.
 * Asynchronous on `stream`. */
int smrt_gemm_bf16(const uint16_t* A, const uint16_t* B, float* C, int32_t M, int32_t N, int32_t K,
                   int32_t lda, int32_t ldb, int32_t ldc, int32_t trans_a, int32_t trans_b,
                   int32_t splits, void* stream);

/* Bandwidth reference: copies `bytes` (a multiple of 16) from src to dst,
 * both device pointers 16-byte aligned, with a plain streaming copy kernel on
 * `stream`.  Used to calibrate byte counters and as the attainable read+write
 * ceiling beside the stream-collide kernel.  Asynchronous. */
int smrt_copy_kernel(const void* src, void* dst, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif
