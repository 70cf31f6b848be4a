/*
 * lbsq.h -- C ABI of the MI355X (gfx950) lattice Boltzmann squirmer library.
 *
 * The library advances the lattice Boltzmann squirmer model of Kuron,
 * Staerk, Burkard, de Graaf and Holm, "A Lattice Boltzmann Model for
 * Squirmers" (arXiv:1903.04799):
 *   - a D3Q19 fluid with the two-relaxation-time collision of Sec.
 *     "Numerical Method", eq. (lb), in a fully periodic box;
 *   - spherical squirmers coupled by moving-wall link bounce-back whose wall
 *     velocity is the rigid-body velocity eq. (vb) plus the surface slip of
 *     eq. (squirmer), B1 (1 + beta e.n)((e.n) n - e);
 *   - momentum-exchange force and torque eqs. (bbforce), (bbtorque) and the
 *     cell-conversion force eq. (consforce), WCA contact repulsion eq. (wca),
 *     and symplectic-Euler rigid-body motion, all on the device.
 *
 * Conventions shared by every call:
 *   - Every call returns an int status: LB_OK (0) or a negative LB_E* code;
 *     lb_strerror() names it.  No C++ exception crosses this boundary.
 *   - Lattice units throughout (grid spacing 1, time step 1).  Cell (i,j,k)
 *     has its centre at (i+1/2, j+1/2, k+1/2).  Linear cell index
 *     x + nx*(y + ny*z), x fastest.  Host arrays are structure-of-arrays.
 *   - Population order (canonical, also the layout of lb_read_populations):
 *       0 rest; 1 +x, 2 -x, 3 +y, 4 -y, 5 +z, 6 -z;
 *       7 (+1,+1,0), 8 (-1,-1,0), 9 (+1,-1,0), 10 (-1,+1,0),
 *       11 (+1,0,+1), 12 (-1,0,-1), 13 (+1,0,-1), 14 (-1,0,+1),
 *       15 (0,+1,+1), 16 (0,-1,-1), 17 (0,+1,-1), 18 (0,-1,+1);
 *     for odd i the opposite direction is i+1.
 *   - The handle is opaque and owned by the caller until lb_destroy.  It is
 *     not thread-safe; distinct handles may be driven concurrently.
 *   - Device memory is owned by the library.  If lb_params.alloc/free are
 *     given, every device allocation goes through them (for example a
 *     framework's caching allocator); otherwise hipMalloc/hipFree are used.
 *     All host buffers passed in are owned by the caller.
 *   - lb_step only enqueues work on the handle's HIP stream and returns.
 *     Calls that hand data back (lb_read_*, lb_force_torque, lb_body_state,
 *     lb_links, lb_audit, lb_sync, lb_save_state) synchronise the stream, and
 *     report errors detected on the device since the previous such call
 *     (LB_EGEOM: overlapping bodies or a body moving a cell or more per step;
 *     LB_ENAN: non-finite populations found by the periodic audit).
 */
#ifndef LBSQ_H
#define LBSQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LB_OK = 0,
    LB_EINVAL = -1,  /* bad argument */
    LB_ENOMEM = -2,  /* device allocation failed */
    LB_EDEVICE = -3, /* HIP runtime error */
    LB_EGEOM = -4,   /* overlapping bodies, body too large for the box, too fast */
    LB_ESTATE = -5,  /* call not allowed in the current state */
    LB_ENAN = -6,    /* non-finite populations detected */
    LB_EBUDGET = -7, /* request exceeds a memory budget */
    LB_ECANCELED = -8 /* request cancelled (lb_server_cancel) */
};

enum { LB_STORAGE_F32 = 0, LB_STORAGE_F16 = 1, LB_STORAGE_BF16 = 2 };
enum { LB_FREE = 0, LB_FIXED = 1, LB_PRESCRIBED = 2 };
enum { LB_OWNER_FLUID = 0, LB_OWNER_WALL = 255 }; /* bodies: id + 1 */
enum { LB_LAYOUT_AUTO = 0, LB_LAYOUT_INPLACE = 1, LB_LAYOUT_AB = 2 };

typedef void *(*lb_alloc_fn)(size_t bytes, void *ctx);
typedef void (*lb_free_fn)(void *ptr, void *ctx);

/* Box and fluid parameters.
 *   nx, ny, nz   box size in cells, each >= 4, nx*ny*nz < 2^32;
 *   nu           kinematic viscosity; lambda_e = 1/(3 nu + 1/2) (the
 *                viscosity relation of Sec. "Numerical Method");
 *   magic        TRT product Lambda = (1/lambda_e - 1/2)(1/lambda_o - 1/2),
 *                3/16 for halfway-exact bounce-back (the paper's printed
 *                "lambda_o lambda_e = 3/16"); lambda_e and lambda_o must lie
 *                in (0, 2);
 *   rho0         reference density (fluid starts at rest with f = w_i rho0);
 *   storage      LB_STORAGE_F32 | _F16 | _BF16: populations are stored as
 *                deviations f_i - w_i rho0 in that type, times 2^scale_log2;
 *                the collision is always computed in FP32;
 *   scale_log2   power-of-two scale of stored deviations (0 for F32/BF16,
 *                typically 14 for F16); 0..20;
 *   wca_sigma, wca_eps   WCA range and strength, eq. (wca);
 *   g            uniform body-force density, a test hook outside the paper's
 *                method (default 0; nonzero only for channel-flow checks);
 *   audit_every  fuse an FP64 mass/momentum audit and non-finite check into
 *                the collision every this many steps (0 = never; every
 *                100 steps costs 0.3% of the step time on MI355X, and is
 *                the Python binding's default);
 *   stream       hipStream_t to run on (NULL = the null stream);
 *   alloc, free, alloc_ctx  optional device allocator pair;
 *   layout       LB_LAYOUT_AUTO (0, the default of a zeroed struct): the
 *                pull layout for boxes of more than 5,500,000 cells (about
 *                176^3), in place below (measured on MI355X: in place wins
 *                at 160^3 and below, pull from 192^3 up);
 *                LB_LAYOUT_INPLACE (1): one population buffer, each step
 *                reads and rewrites it in place (half the memory; the
 *                faster form while the buffer fits the 256 MB last-level
 *                cache); LB_LAYOUT_AB (2): two buffers, each step pulls
 *                from one and writes the other (the faster form for boxes
 *                whose populations stream from HBM).  Results agree bit
 *                for bit.  A saved state records the resolved layout and
 *                restores only into a handle of the same one. */
typedef struct lb_params {
    int nx, ny, nz;
    double nu, magic, rho0;
    int storage;
    int scale_log2;
    double wca_sigma, wca_eps;
    double g[3];
    int audit_every;
    void *stream;
    lb_alloc_fn alloc;
    lb_free_fn free;
    void *alloc_ctx;
    int layout;
} lb_params;

/* One spherical squirmer, eq. (squirmer) with beta = B2/B1.
 *   pos   centre, lattice units, any real value (wrapped into the box);
 *   e     orientation (normalised by the library; LB_EINVAL if zero);
 *   R     radius (> 0.5); the box must satisfy 2*(ceil(R)+3)+1 <= min(n);
 *   B1, beta  slip amplitude and dipolarity; B1 = 0 is a no-slip sphere;
 *   mode  LB_FREE (moves under F and T), LB_FIXED (never moves; F and T are
 *         still measured), LB_PRESCRIBED (moves with the given v, w);
 *   v, w  initial (FREE) or imposed (PRESCRIBED) velocity and angular
 *         velocity; |v| must stay below one cell per step;
 *   rho_p particle density for the mass m = rho_p 4/3 pi R^3 and moment of
 *         inertia I = 2/5 m R^2 (<= 0 means rho0).                           */
typedef struct lb_squirmer {
    double pos[3], e[3];
    double R, B1, beta;
    int mode;
    double v[3], w[3];
    double rho_p;
} lb_squirmer;

typedef struct lb_sim lb_sim;

/* Allocate a periodic box at rest.  LB_EINVAL for a dimension < 4, nu <= 0,
 * relaxation rates outside (0, 2) or an unknown storage type. */
int lb_create(const lb_params *p, lb_sim **out);

/* Static no-slip walls (bounce-back with zero wall velocity, the no-slip
 * rule of Sec. "Numerical Method"): solid[c] != 0 marks cell c as wall.  n
 * must equal nx*ny*nz.  Only before the first step and before any body.
 * A mask with walls takes 4 more bytes of device memory per cell (each
 * cell's wall links) and a list of the groups of 256 cells that hold a
 * non-wall cell (groups of walls alone are never streamed); a mask without
 * walls releases both.  Cells are numbered x fastest, so a channel along x
 * keeps wall and fluid cells in separate cache lines and moves least
 * memory.  LB_ENOMEM if the masks cannot be allocated.                    */
int lb_set_static_mask(lb_sim *s, const uint8_t *solid, size_t n);

/* Add a body (see lb_squirmer); *id receives its index (0, 1, ...).  The
 * cells inside it become solid at once (no conversion force at t = 0).
 * LB_EGEOM if it overlaps a wall or another body or is too large for the
 * box; LB_ESTATE after the first step. At most 252 bodies.               */
int lb_add_squirmer(lb_sim *s, const lb_squirmer *sq, int *id);

/* Enqueue nsteps time steps on the handle's stream.  Each step: streaming
 * with bounce-back and momentum exchange, TRT collision, rigid-body update
 * from the force and torque (momentum exchange, WCA, and the conversion
 * force of the previous move), then geometry at the new positions and cell
 * conversion.  Between steps the cell owners match the body positions.     */
int lb_step(lb_sim *s, int nsteps);

/* Advance n distinct handles by nsteps each, together: each step is one
 * fluid launch and one geometry launch covering all of them, enqueued on the
 * stream of sims[0] after the work already queued on every handle's stream
 * (the other streams then wait for the batch).  Each handle gives the same
 * result, bit for bit, that lb_step would give it alone.  Handles that
 * cannot share a launch (different storage, a body force g, a fused audit,
 * kernel timing, more than 8 bodies, more than 64 handles) are stepped one
 * after the other instead.  LB_EINVAL if a handle is NULL or repeated.     */
int lb_step_batch(lb_sim *const *sims, int n, int nsteps);

/* Block until the handle's queued work is done; reports device errors.   */
int lb_sync(lb_sim *s);

/* Density, velocity (u[k*N + c]) and owner (0 fluid, id+1 body, 255 wall;
 * may be NULL) at the current time, FP64 host buffers of N, 3N and N.
 * Solid cells get rho = 0 and u = 0.  u = sum f c / rho (with a body force
 * g: (sum f c - g/2)/rho, the half-step velocity).                          */
int lb_read_fields(lb_sim *s, double *rho, double *u, uint8_t *owner);

/* For callers that cannot allocate device memory (code around HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * readout as lb_read_fields, same arguments, layout and results (bit for
 * bit), with no device allocation and no call of the handle's allocator.
 * The fields pass through a fixed 16 MiB device array per GPU, held until
 * the process ends, in chunks of 508,160 cells; any box size is read.
 * Every call on one GPU shares that array: calls from several threads are
 * serialised by a per-device lock (overlapping calls would race on it), and
 * each returns only after its last copy out of the array has ended.
 * LB_EINVAL for a NULL handle, rho or u; LB_EDEVICE if the array's device
 * address cannot be obtained or a launch or copy fails.                     */
int lb_read_fields_noalloc(lb_sim *s, double *rho, double *u, uint8_t *owner);

/* Hydrodynamic force and torque on body id from the last completed step:
 * momentum exchange eqs. (bbforce), (bbtorque) plus conversion eq.
 * (consforce).  These are the values the integrator used, minus WCA.       */
int lb_force_torque(lb_sim *s, int id, double F[3], double T[3]);

/* Same, split: momentum exchange (Fbb, Tbb) and conversion (Fc, Tc).       */
int lb_force_parts(lb_sim *s, int id, double Fbb[3], double Tbb[3], double Fc[3], double Tc[3]);

/* FP64 rigid-body state of body id after the last completed step; Fwca is
 * the WCA force of that step. Any pointer may be NULL.                     */
int lb_body_state(lb_sim *s, int id, double pos[3], double e[3], double v[3], double w[3],
                  double Fwca[3]);

/* The current boundary-link set {(c, i, o) : cell c fluid and cell
 * c - c_i solid with owner o}, sorted by (c, i).  If cap < count, nothing
 * is copied, *n receives the count and LB_EINVAL is returned.              */
int lb_links(lb_sim *s, uint32_t *cell, uint8_t *dir, uint8_t *owner, size_t cap, size_t *n);

/* Populations f_i (absolute, FP64, canonical order, f[i*N + c]); solid
 * cells read 0 and are ignored on write.  Writing replaces the fluid state. */
int lb_read_populations(lb_sim *s, double *f);
int lb_write_populations(lb_sim *s, const double *f);

/* FP64 total mass sum f and momentum sum f c over fluid cells.            */
int lb_audit(lb_sim *s, double *mass, double P[3]);

/* Number of fluid cells and of completed steps.                           */
int lb_info(lb_sim *s, uint64_t *n_fluid, int64_t *steps);

/* Checkpoint: the complete state (populations in storage format, cell
 * owners, bodies, step count) as an opaque byte blob. lb_state_size gives
 * its size; lb_load_state accepts only a blob from a handle created with
 * the same lb_params and resumes bit for bit.                              */
int lb_state_size(lb_sim *s, size_t *bytes);
int lb_save_state(lb_sim *s, void *buf, size_t bytes);
int lb_load_state(lb_sim *s, const void *buf, size_t bytes);

/* Kernel timing for measurement: when enabled, every launch of the
 * fluid-update kernel (streaming, bounce-back and collision of every fluid
 * cell) made by lb_step carries a pair of HIP events that the launch stamps
 * with its own start and end; lb_kernel_time returns the summed duration
 * (ms) and launch count since it was enabled.  Timing changes no result;
 * the events cost host time per step, so time the steps themselves in a
 * separate pass.  lb_kernel_time returns LB_EDEVICE (and drops the
 * pending events) if an elapsed time cannot be read.                      */
int lb_kernel_timing(lb_sim *s, int enable);
int lb_kernel_time(lb_sim *s, double *ms, int64_t *launches);

int lb_destroy(lb_sim *s);
const char *lb_strerror(int code);

/* ------------------------------------------------------------------------
 * Serving: a stream of independent squirmer simulations (requests) of
 * different box sizes, radii and beta, kept resident in one device-memory
 * arena and advanced together with continuous batching.
 *
 *   - Admission is first come, first served, while fewer than max_active
 *     requests are resident and the next one fits in the arena of
 *     budget_bytes; the rest wait in the queue.
 *   - The resident requests advance in chunks of chunk_steps steps; each
 *     step of a chunk is one batched fluid launch and one batched geometry
 *     launch over all of them (captured once as a HIP graph per set of
 *     resident requests when use_graph is set).  Requests join and leave
 *     between chunks, so new arrivals overlap on the device with the work
 *     already running, and a finished request's memory returns to the arena.
 *   - Every request ends after exactly its nsteps steps with the result it
 *     would have had as a handle of its own stepped by lb_step (same
 *     kernels, bit for bit).
 *   - Up to two chunks are queued on the device at a time; lb_server_progress
 *     retires finished chunks, reads the results of the requests they
 *     completed, admits queued requests and enqueues the next chunk.
 * The server is not thread-safe.  Times are seconds on the server's clock
 * (steady, from lb_server_create).                                        */

enum { LB_REQ_MAXBODY = 8, LB_SERVER_MAXACTIVE = 64 };

typedef struct lb_server lb_server;

/* budget_bytes  device memory of the arena for resident requests (>= 2^20);
 * max_active    resident requests at most, 1..64;
 * chunk_steps   steps per chunk, 1..100000;
 * use_graph     replay each chunk as a HIP graph (0: plain launches);
 * storage, scale_log2, wca_sigma, wca_eps  as in lb_params, for every
 *               request (nu comes with each request, rho0 = 1, magic 3/16);
 * stream        hipStream_t of the batched steps (NULL: the server creates
 *               a non-blocking stream);
 * layout        population layout of every request: LB_LAYOUT_INPLACE or
 *               LB_LAYOUT_AB as in lb_params; LB_LAYOUT_AUTO (0) takes the
 *               pull layout, since a batch of resident requests streams
 *               from HBM (the pull layout takes twice the population memory
 *               of each request from the budget).                         */
typedef struct lb_server_params {
    size_t budget_bytes;
    int max_active;
    int chunk_steps;
    int use_graph;
    int storage, scale_log2;
    double wca_sigma, wca_eps;
    void *stream;
    int layout;
} lb_server_params;

/* One request: a periodic nx x ny x nz box at rest with viscosity nu and
 * nbody (0..8) bodies, run for nsteps (>= 0) steps.  tag is handed back
 * with the result.                                                        */
typedef struct lb_request {
    int nx, ny, nz;
    double nu;
    int nbody;
    lb_squirmer body[LB_REQ_MAXBODY];
    int64_t nsteps;
    uint64_t tag;
} lb_request;

/* Result of a request: status LB_OK or the error that ended it (for example
 * LB_EGEOM for overlapping bodies); body states and hydrodynamic force and
 * torque after the last step (as lb_body_state and lb_force_torque); the
 * FP64 fluid mass of the final state (lb_audit); the fluid cells at
 * admission (the unit of the server's cell-update count); the server times
 * of submission, admission and completion.                                */
typedef struct lb_result {
    uint64_t ticket, tag;
    int status;
    int nbody;
    int64_t steps;
    uint64_t fluid_cells;
    double pos[LB_REQ_MAXBODY][3], e[LB_REQ_MAXBODY][3], v[LB_REQ_MAXBODY][3], w[LB_REQ_MAXBODY][3];
    double F[LB_REQ_MAXBODY][3], T[LB_REQ_MAXBODY][3];
    double mass;
    double t_submit, t_admit, t_done;
} lb_result;

/* Counters since creation: lattice updates of fluid cells, chunks, graphs
 * built, requests completed, and the arena's bytes in use now.            */
typedef struct lb_server_stats {
    uint64_t cell_updates;
    uint64_t chunks;
    uint64_t graphs;
    uint64_t completed;
    size_t arena_in_use;
} lb_server_stats;

/* LB_EINVAL for out-of-range parameters (checked before any device call),
 * LB_ENOMEM if the arena cannot be allocated.                             */
int lb_server_create(const lb_server_params *p, lb_server **out);

/* Queue a request; *ticket (may be NULL) identifies its result.  LB_EINVAL
 * for a malformed request, LB_EBUDGET if it can never fit in the arena.   */
int lb_server_submit(lb_server *sv, const lb_request *rq, uint64_t *ticket);

/* Retire finished chunks, admit, enqueue the next chunk; with wait != 0
 * first block until the oldest queued chunk is done.  *active and *queued
 * (may be NULL) receive the resident and waiting request counts.          */
int lb_server_progress(lb_server *sv, int wait, int *active, int *queued);

/* Cancel a request.  A queued request ends at once; a resident one leaves
 * the batch at once and ends when the chunks already queued with it have
 * run (its device memory is released only then).  Either way its result
 * carries status LB_ECANCELED and the steps it ran.  LB_EINVAL for a ticket
 * the server never issued, LB_ESTATE for a request that has already ended
 * or is in its final chunk (its result comes as usual).                   */
int lb_server_cancel(lb_server *sv, uint64_t ticket);

/* Move up to cap completed results to out (oldest first); *n receives how
 * many.                                                                    */
int lb_server_results(lb_server *sv, lb_result *out, int cap, int *n);

int lb_server_stats_get(lb_server *sv, lb_server_stats *st);
int lb_server_clock(lb_server *sv, double *t);

/* Wait for the queued chunks, drop every request still resident or
 * queued, and free the arena.                                             */
int lb_server_destroy(lb_server *sv);

#ifdef __cplusplus
}
#endif
#endif /* LBSQ_H */
