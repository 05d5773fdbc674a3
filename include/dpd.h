/*
 * dpd.h -- C ABI of the MI355X (gfx950) DPD hot-path library (libdpd.so).
 *
 * The library implements one time step of dissipative particle dynamics as
 * described by Tang & Karniadakis, "Accelerating Dissipative Particle
 * Dynamics Simulations on GPUs" (arXiv 1311.0402): cell binning and particle
 * reordering (Sec. 3.2), an ordered neighbour list (Sec. 3.3), the pairwise
 * conservative + dissipative + random force (Sec. 2, Eqs (2)-(8)) with a
 * pair Gaussian regenerated from particle tags, step and seed (Sec. 3.5),
 * and the velocity-Verlet integration phases of Algorithm 1.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory    Every array argument is DEVICE memory owned by the caller; the
 *           library never allocates or frees device memory.  Scratch space
 *           is a caller-provided workspace sized by dpd_workspace_bytes().
 *           Parameter blocks (dpd_params, dpd_state, ...) are HOST memory
 *           and are read during the call only.
 * Layout    Positions, velocities and forces are structure of arrays
 *           double[3][n] (all x, then all y, then all z).  Tags are uint32
 *           (a particle's identity, invariant under reordering), types
 *           uint8 (< n_types <= DPD_MAX_TYPES).  Indices are int32 (n and
 *           the neighbour count must stay below 2^31).
 * Streams   Every enqueuing call takes a hipStream_t (as void*, NULL = the
 *           default stream), is asynchronous, performs no host-device
 *           synchronisation and no allocation, so it may be captured in a
 *           HIP graph.
 * Errors    Every call returns a dpd_status.  Argument errors are detected
 *           before anything is enqueued (nothing is launched).  Conditions
 *           that only the device can see (neighbour-list overflow,
 *           non-finite totals, broken bond tables) are OR-ed as
 *           DPD_STATUS_* bits into the caller's device int32 *d_status,
 *           which the caller reads after synchronising.  dpd_last_error()
 *           returns a thread-local message for the last failing call.
 *           Nothing throws across this boundary and nothing aborts.
 * Geometry  Periodic box [0, L_x) x [0, L_y) x [0, L_z).  The separation of
 *           two particles is the minimum image of r_i - r_j, computed by
 *           subtracting first and then shifting by one box length; the
 *           squared distance is fma(dz, dz, fma(dy, dy, dx * dx)).  Cells
 *           have n_c = floor(L / r_list) per side, reduced while the side
 *           L / n_c is below r_list (1 + 2^-40); n_c must be in [3, 1023].
 */
#ifndef DPD_H
#define DPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPD_MAX_TYPES 8

typedef enum dpd_status {
    DPD_OK = 0,
    DPD_EINVAL = -1,        /* bad argument (null pointer, size, parameter) */
    DPD_ECAPACITY = -2,     /* a caller buffer is too small                  */
    DPD_EHIP = -3,          /* the HIP runtime reported an error             */
    DPD_EUNSUPPORTED = -4   /* valid request this build does not implement   */
} dpd_status;

/* bits of the device status word */
#define DPD_STATUS_NLIST_OVERFLOW 1   /* neighbour list exceeded its capacity   */
#define DPD_STATUS_NONFINITE      2   /* a step produced non-finite totals      */
#define DPD_STATUS_BAD_BOND       4   /* a bond partner tag has no particle     */
#define DPD_STATUS_HALO_OVERFLOW  8   /* a send list or ghost range did not fit */

typedef enum dpd_precision {
    DPD_FP64 = 0,   /* pair arithmetic in FP64                                 */
    DPD_MIXED = 1   /* pair arithmetic in FP32 on cell-relative coordinates,
                       compensated FP32 sums, FP64 forces, state, integration
                       and reductions                                          */
} dpd_precision;

/* Physical and numerical parameters (host memory). */
typedef struct dpd_params {
    double box[3];          /* periodic box lengths                             */
    double r_c;             /* force cutoff, Eqs (3)-(6)                         */
    double skin;            /* neighbour radius is r_c + skin (>= 0); dpd_step
                               rebuilds lists on displacement when > 0      */
    double dt;              /* time step; F^R scales as dt^-1/2 (Eq (5))        */
    double lambda;          /* velocity-prediction factor of the integrator:
                               F^D sees v + lambda dt F (0.5 = half-step v)     */
    double s;               /* weight exponent, w_R = (1 - r/r_c)^s (Eq (8))    */
    int32_t n_types;        /* 1 .. DPD_MAX_TYPES                               */
    int32_t reserved0;
    double a[DPD_MAX_TYPES * DPD_MAX_TYPES];      /* a_ij, row-major, symmetric  */
    double gamma[DPD_MAX_TYPES * DPD_MAX_TYPES];  /* gamma_ij, symmetric         */
    double sigma[DPD_MAX_TYPES * DPD_MAX_TYPES];  /* sigma_ij, symmetric (Eq (9)
                                                     ties it to gamma; the ABI
                                                     takes it as given)         */
    uint64_t seed;          /* global seed of the pair Gaussian                  */
    double body_g;          /* body force along x: +g where y < body_split,
                               -g elsewhere (0 = none)                           */
    double body_split;
    double bond_k;          /* harmonic bonds F = -k (r - r0) e                  */
    double bond_r0;
    const int32_t* bond_partner;  /* DEVICE int32[2 n] indexed by tag: up to two
                                     partner tags per particle, -1 = none; NULL
                                     = no bonds.  Requires tags to be a
                                     permutation of 0..n-1.                      */
} dpd_params;

/* One system's particle arrays (device pointers; host struct). */
typedef struct dpd_state {
    int32_t n;
    int32_t reserved0;
    double* x;              /* [3][n], each component in [0, L)                 */
    double* v;              /* [3][n]                                            */
    double* f;              /* [3][n]                                            */
    uint32_t* tag;          /* [n]                                               */
    uint8_t* type;          /* [n]                                               */
} dpd_state;

/* Cell list of a reordered state (device pointers; host struct). */
typedef struct dpd_cells {
    int32_t* cell_start;    /* [n_cells + 1]: first particle of every cell, cells
                               in ascending Morton rank; last entry = n          */
    uint32_t* cell_xyz;     /* [n]: cell of each sorted particle,
                               cx | cy << 10 | cz << 20                          */
    int32_t* perm;          /* [n]: sorted index -> input index                  */
    int32_t* idx_of_tag;    /* [n]: tag -> sorted index (required with bonds,
                               else nullable)                                    */
} dpd_cells;

/* Neighbour list in CSR form (device pointers; host struct). */
typedef struct dpd_nlist {
    int64_t capacity;       /* entries available in index[]                     */
    int32_t* offset;        /* [n + 1]: row i is index[offset[i] .. offset[i+1]) */
    int32_t* index;         /* [capacity]: neighbours, each row strictly ascending */
} dpd_nlist;

/* ---------------------------------------------------------------------------
 * Queries (host only, nothing enqueued)
 * ------------------------------------------------------------------------- */

/* Message of the last failing call on this thread ("" if none). */
const char* dpd_last_error(void);

/* Library version string. */
const char* dpd_version(void);

/* How the force pass walks the list (a process-wide host setting).  The
 * pair terms of Eqs (2)-(5) are antisymmetric, f_ji = -f_ij, so a pair of
 * two particles inside the same chunk of 64 consecutive sorted particles
 * (chunks counted from each system's first particle) can be evaluated once,
 * from the lower particle's row, with its negated force going to the upper
 * particle; the list rows stay full either way.
 *   mode 0: every list entry is evaluated (each pair from both rows);
 *   mode 1: pairs inside a chunk once, in both precisions;
 *   mode 2 (default): pairs inside a chunk once in the FP64 form, every
 *           entry in the mixed form (the faster choice for each on MI355X).
 * The modes differ only in the order of each particle's sums; each is
 * deterministic.  It applies to launches enqueued afterwards (a batch's
 * cached step graph is captured again).  Returns the previous mode, or
 * DPD_EINVAL for another value. */
int dpd_set_pair_evaluation(int32_t mode);

/* Which neighbour-list builder single-system calls (dpd_build_neighbors,
 * dpd_step) use, a process-wide host setting; every builder writes the same
 * ordered rows (Sec. 3.3.2: a particle's neighbours in the ascending order
 * of their cells' ranks over its 27 stencil cells, by index within a cell).
 *   kind 0 (default): one workgroup per 8x4x4-cell tile, the tile's
 *          neighbourhood staged in LDS;
 *   kind 1: one wave per 2x2x2-cell block with ballot compaction (its slab
 *          entries carry no stencil code);
 *   kind 2: one lane per particle over global memory.
 * Batches choose theirs with dpd_batch_set_tiles.  Applies to calls
 * enqueued afterwards.  Returns the previous kind, or DPD_EINVAL for
 * another value. */
int dpd_set_list_builder(int32_t kind);

/* Cells per side for these parameters (rule in the header comment).
 * Returns DPD_EINVAL when the box holds fewer than 3 or more than 1023 cells
 * per side. */
int dpd_cell_grid(const dpd_params* p, int32_t nc[3]);

/* Bytes of workspace needed by any call below for n particles at this
 * precision (0 on invalid arguments).  One workspace serves every entry
 * point; it must be 256-byte aligned. */
size_t dpd_workspace_bytes(const dpd_params* p, int32_t n, int32_t precision);

/* ---------------------------------------------------------------------------
 * Hot-path calls
 * ------------------------------------------------------------------------- */

/* Binning and reordering (Sec. 3.2.2 and 3.2.3).
 * Each particle of `in` is assigned the cell c_k = min(n_c,k - 1,
 * trunc(x_k * n_c,k / L_k)); cells are ranked along the Morton (Z) curve
 * with bit b of c_x at 3b, c_y at 3b+1, c_z at 3b+2; particles are written to
 * `out` in ascending (cell rank, tag) order.  in and out must not overlap.
 * out->f is not touched.  cells receives cell_start, cell_xyz, perm and
 * (if non-NULL) idx_of_tag.  When x32 / v32 are non-NULL they receive
 * packed FP32 copies, one float4 per sorted particle ([n][4], 16-byte
 * aligned): x32[i] = ((float)(x_k - c_k L_k / n_c,k) for k = x, y, z -- the
 * offset inside the particle's cell --, tag bits) and v32[i] = ((float)v,
 * type as uint32 bits).  The neighbour list needs x32; the mixed-precision
 * force needs both. */
int dpd_bin_reorder(const dpd_params* p, const dpd_state* in, dpd_state* out,
                    dpd_cells* cells, float* x32, float* v32,
                    void* ws, size_t ws_bytes, void* stream);

/* Ordered neighbour list (Sec. 3.3.2).
 * For a state produced by dpd_bin_reorder (x32 = its FP32 in-cell offsets):
 * row i lists every j != i with |r_ij|^2 < (r_c + skin)^2 (the FP64 rule of
 * the header comment, bit for bit) in strictly ascending j.  One 64-lane
 * wavefront per 2x2x2 block of cells scans the surrounding cells in
 * ascending rank; an FP32 pre-test on the offsets decides all pairs outside
 * a narrow band around the cutoff and the FP64 rule decides inside it;
 * insertion points come from a wavefront ballot and a lane prefix count (no
 * atomics, deterministic).  If the rows need more than nl->capacity entries,
 * DPD_STATUS_NLIST_OVERFLOW is set in *d_status, offset[] still holds the
 * required row sizes (offset[n] = the total needed) and index[] is not
 * written. */
int dpd_build_neighbors(const dpd_params* p, const dpd_state* sorted, const dpd_cells* cells,
                        const float* x32, dpd_nlist* nl, int32_t* d_status,
                        void* ws, size_t ws_bytes, void* stream);

/* Pairwise DPD forces (Sec. 2, Eqs (2)-(8)) plus bonds (Sec. 4.5) and the
 * body force (Sec. 4.2), at time-step counter `step`.
 * For every listed pair with |r_ij| < r_c:
 *   F_ij = (a w_C - gamma w_D (e.v_ij) + sigma w_R xi_ij / sqrt(dt)) e_ij,
 *   w_C = 1 - r/r_c, w_R = w_C^s, w_D = w_R^2, e_ij = r_ij / r, v_ij from
 *   `v` (the predicted velocity), and
 *   xi_ij = sqrt(-2 ln u1) cos(2 pi u2), (u1, u2) = ((w0 + 1/2) 2^-32,
 *   w1 2^-32), (w0..w3) = Philox4x32-10(counter = (min tag, max tag,
 *   step low word, step high word), key = (seed low word, seed high word)).
 * f_out[i] = the sum over i's row (a fixed reduction tree over the row's
 * list entries: deterministic for a given list), plus bonds and body force.
 * DPD_MIXED evaluates the pair terms in FP32 from x32 / v32 / cells->cell_xyz
 * (as written by dpd_bin_reorder) and sums them with compensated FP32;
 * DPD_FP64 ignores x32 / v32.  pe_out (nullable, [n]) gets each particle's
 * half of its pair and bond potential energies (1/2 a r_c w_C^2 per pair,
 * 1/2 k (r - r0)^2 per bond).  stats (nullable, device double[2]) gets the
 * total potential energy and the number of unique pairs inside r_c.
 * d_status may be NULL when no bonds are present. */
int dpd_forces(const dpd_params* p, int32_t precision, const dpd_state* sorted,
               const dpd_cells* cells, const float* x32, const float* v32,
               const dpd_nlist* nl, uint64_t step, double* f_out, double* pe_out,
               double* stats, int32_t* d_status,
               void* ws, size_t ws_bytes, void* stream);

/* dpd_forces without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * dpd_forces; the force pass's per-workgroup partials of `stats` (potential
 * energy, pair count) go to a static device array of the library (8,192 x 2
 * doubles = 128 KiB per device, held until the process ends) instead of the
 * caller's workspace, so nothing is allocated.  The array's device address
 * is looked up on the first call on each device.  Limit: the force grid
 * never exceeds 8,192 workgroups, so every n fits; a larger grid would be
 * rejected with DPD_ECAPACITY.  Every call on a device shares that device's
 * array (each call overwrites the partials it reads, nothing needs to start
 * at zero): calls whose stats passes overlap on one device, on different
 * streams or from different threads, race. */
int dpd_forces_noalloc(const dpd_params* p, int32_t precision, const dpd_state* sorted,
                       const dpd_cells* cells, const float* x32, const float* v32,
                       const dpd_nlist* nl, uint64_t step, double* f_out, double* pe_out,
                       double* stats, int32_t* d_status, void* stream);

/* n_steps time steps of Algorithm 1 on one system:
 *   v_h = v + dt/2 F;  x <- x + dt v_h, wrapped into [0, L);
 *   v~  = v + lambda dt F (= v_h when lambda = 1/2);
 *   reorder, rebuild the list, F <- F(x, v~, step + 1);
 *   v   = v_h + dt/2 F;  step <- step + 1.
 * With p->skin = 0 the cell and neighbour lists are rebuilt every step.
 * With p->skin > 0 (Sec. 3.3: lists of radius r_c + skin, rebuilt every few
 * steps) the first step of the call rebuilds them; each later step rebuilds
 * (reorders and builds the list) only when some particle has moved more than
 * skin / 2 from where the last rebuild saw it, which keeps every pair inside
 * r_c in the list; otherwise the state keeps its order and the step goes
 * straight to the forces (which skip listed pairs at r >= r_c: the FP64
 * separation decides in the FP64 form, the FP32 one in the mixed form).  The
 * decision is taken on the device, step by step.  cells->perm then describes
 * the last reorder of the call.
 * On entry st->f must hold the forces of the current state (e.g. from
 * dpd_forces at the current step).  x32 (packed FP32 in-cell offsets,
 * float4 [n], see dpd_bin_reorder) is always required; v32 (float4 [n])
 * only for DPD_MIXED.  *d_step (device uint64) is the step
 * counter: read at every step and incremented on the device, so a captured
 * graph can be replayed.  On exit st holds the reordered state and
 * cells / nl describe it (within a call the force pass reads each step's
 * rows from the workspace; nl's CSR index is written for the last step
 * only, and its capacity is checked every step; with bonds, the force pass
 * finds partners through sorted partner indices kept in the workspace and
 * cells->idx_of_tag is written at the first and the last step).  d_reductions (nullable, device double[n_steps][8])
 * receives per step: P_x, P_y, P_z, sum |v|^2, potential energy, unique
 * pairs, sum |v - v_mean|^2 / (3 (n - 1)) (k_B T), and 1 when the step
 * rebuilt the cell and neighbour lists (always with skin 0), else 0.
 * phase_events (nullable): hipEvent_t[6 * n_steps], created by the caller;
 * for step k, events 6k .. 6k+5 are recorded on `stream` before the first
 * integration phase, after it, after reordering, after the neighbour list,
 * after the forces and after the second phase and statistics, so the
 * caller can time each phase of every step.  (The second phase of a step
 * and the first phase of the next run as one pass over the state and are
 * timed with the next step's first phase; the last step's second phase
 * runs alone.) */
int dpd_step(const dpd_params* p, int32_t precision, dpd_state* st, int32_t n_steps,
             uint64_t* d_step, double* d_reductions, dpd_cells* cells, dpd_nlist* nl,
             float* x32, float* v32, int32_t* d_status, void* const* phase_events,
             void* ws, size_t ws_bytes, void* stream);

/* Vector-Jacobian product of the deterministic force map (xi and the pair
 * set held fixed) for an upstream gradient g = dL/dF ([3][n]):
 *   x_bar_i = sum_j (df_ij/dr_ij)^T (g_i - g_j)   (plus bond terms),
 *   v_bar_i = sum_j (df_ij/dv_ij)^T (g_i - g_j),
 *   a_bar[t][u] = dL/da_tu for the symmetric parameter (both entries equal),
 *   gamma_bar[t][u] likewise,
 * evaluated at the same (sorted state, list, step) as dpd_forces (FP64).
 * a_bar / gamma_bar are device double[n_types * n_types].  With accumulate
 * != 0 all four outputs are added to instead of overwritten. */
int dpd_forces_backward(const dpd_params* p, const dpd_state* sorted, const dpd_cells* cells,
                        const dpd_nlist* nl, uint64_t step, const double* grad_f,
                        double* grad_x, double* grad_v, double* grad_a, double* grad_gamma,
                        int32_t accumulate, void* ws, size_t ws_bytes, void* stream);

/* Reverse of one dpd_step time step (lambda = 1/2 only), for trajectory
 * gradients with ξ and the pair sets held fixed.  st / cells / nl are the
 * state AFTER the step (as dpd_step leaves them: reordered x', v', F', and
 * cells->perm mapping its order to the order before the step), `step` its
 * counter value.  The forward step is
 *   v_h = v + dt/2 F;  x' = x + dt v_h;  F' = F(x', v_h, step);
 *   v' = v_h + dt/2 F';  then reordering by perm.
 * Given the adjoints (gx_in, gv_in, gf_in) of (x', v', F') in the new order,
 * writes the adjoints (gx_out, gv_out, gf_out) of (x, v, F) in the order
 * before the step, and ADDS the step's contribution to grad_a / grad_gamma
 * (symmetric-parameter gradients, device double[n_types^2]).  v_h is taken
 * as v' - dt/2 F' (equal to the forward value up to rounding).  Outputs must
 * not alias inputs; all arrays [3][n] device FP64.
 * Returns DPD_EUNSUPPORTED for lambda != 1/2. */
int dpd_step_backward(const dpd_params* p, const dpd_state* st, const dpd_cells* cells,
                      const dpd_nlist* nl, uint64_t step, const double* gx_in, const double* gv_in,
                      const double* gf_in, double* gx_out, double* gv_out, double* gf_out,
                      double* grad_a, double* grad_gamma, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Border determination and ghost exchange (Sec. 3.6, Algorithm 6)
 *
 * In a spatial decomposition each GPU owns a brick [lo, hi) and sends
 * copies of the particles within `width` (r_c + skin) of each face to the
 * neighbour across it, which keeps them as ghosts.  These calls are the one
 * GPU's part of that exchange: flags, a multi-block scan and a compaction
 * that produce the six send lists (after each reorder, since indices
 * change), then packing of the listed particles into ghost records, and
 * unpacking of received records into the ghost range of a state.  Moving
 * the records between GPUs (e.g. RCCL send / recv of the record buffers)
 * is the caller's.  Exchanging the x faces first, then the y faces with the
 * x ghosts included, then the z faces with all ghosts, reaches the edge and
 * corner neighbours too.
 * ------------------------------------------------------------------------- */

/* One ghost record (56 bytes). */
typedef struct dpd_ghost {
    double x[3];            /* position plus the face's shift (the periodic
                               image the receiving neighbour sees)           */
    double v[3];
    uint32_t tag;
    uint32_t type;
} dpd_ghost;

/* Workspace bytes of dpd_border_lists for n particles (0 for n < 0). */
size_t dpd_border_workspace_bytes(int32_t n);

/* Send lists of the faces selected by face_mask (bit f, f = 2 d + s for axis
 * d = 0, 1, 2 and s = 0 the low face, 1 the high face) of the brick
 * [lo, hi) (host double[3] each, lo < hi), over the st->n particles of st
 * (ghosts included when the caller appended some): face f lists, in
 * ascending index order, every particle with x_d < lo_d + width (s = 0) or
 * x_d >= hi_d - width (s = 1).  send_offset (device int32[7]) receives the
 * exclusive offsets of the six lists in send_index (unselected faces are
 * empty; send_offset[6] = the total).  When the total exceeds capacity,
 * send_index is not written and DPD_STATUS_HALO_OVERFLOW is set in
 * *d_status (send_offset still holds the sizes).  ws: device memory of
 * dpd_border_workspace_bytes(st->n) bytes, 256-byte aligned. */
int dpd_border_lists(const dpd_state* st, const double lo[3], const double hi[3], double width, int32_t face_mask,
                     int32_t* send_offset, int32_t* send_index, int64_t capacity, int32_t* d_status, void* ws,
                     size_t ws_bytes, void* stream);

/* One record per send-list entry r (send lists and offsets from
 * dpd_border_lists on the same state): records[r] = (x_j + shift[f],
 * v_j, tag_j, type_j), j = send_index[r], f its face; shift is host
 * double[6][3] (e.g. +L_d for the low face and -L_d for the high face of a
 * brick that spans the periodic box along d).  records: device
 * dpd_ghost[capacity].  Nothing is written when the lists overflowed; an
 * entry that is no index of st sets DPD_STATUS_HALO_OVERFLOW. */
int dpd_border_pack(const dpd_state* st, const int32_t* send_offset, const int32_t* send_index, int64_t capacity,
                    const double shift[18], dpd_ghost* records, int32_t* d_status, void* stream);

/* Unpacks records[0 .. *d_count) (device count, e.g. send_offset + 6 of the
 * sender) into dst at indices first .. first + count - 1: x, v, tag, type.
 * dst->n is the size of dst's arrays (owned particles plus room for
 * ghosts).  A count above capacity or past dst->n sets
 * DPD_STATUS_HALO_OVERFLOW and writes nothing. */
int dpd_border_unpack(const dpd_ghost* records, const int32_t* d_count, int64_t capacity, dpd_state* dst,
                      int32_t first, int32_t* d_status, void* stream);

/* ---------------------------------------------------------------------------
 * The paper's numerics as A/B variants (Sec. 3.5, Algorithms 4 and 5,
 * Table 3): the TEA hash on per-particle signatures and reduced-branch
 * logarithm, cosine and power functions, beside the device library the
 * force kernels call.  Study entry points: the force kernels keep
 * Philox4x32-10 and the device library.
 * ------------------------------------------------------------------------- */

typedef enum dpd_math_fn {
    DPD_FN_LOG = 0,          /* ln a, device library                                */
    DPD_FN_FASTLOG = 1,      /* ln a (a > 0, normal): exponent from the bits, the
                                mantissa's log by the atanh power series          */
    DPD_FN_COS2PI = 2,       /* cos(2 pi a), device library (cospi)                 */
    DPD_FN_FASTCOS2PI = 3,   /* cos(2 pi a) for a in [0, 1): symmetry folding and
                                the cos / sin power series on [0, pi/4]           */
    DPD_FN_POW = 4,          /* a^b, device library                                 */
    DPD_FN_FASTPOW = 5       /* a^b (a > 0 normal, result normal) as 2^N 2^r with
                                r = b log2 a - N, |r| <= 1/2                      */
} dpd_math_fn;

/* out[i] = fn(a[i], b[i]) for i < n (b read by the power functions only,
 * nullable otherwise); device arrays. */
int dpd_math_eval(int32_t fn, int64_t n, const double* a, const double* b, double* out, void* stream);

/* One wavefront evaluates a chain of `chain` dependent calls of fn per lane
 * (each argument an affine map of the previous result); d_cycles (device
 * int64[1]) receives the shader-clock ticks of the chain, d_sink (device
 * double[64]) the lanes' last values. */
int dpd_math_latency(int32_t fn, int32_t chain, int64_t* d_cycles, double* d_sink, void* stream);

/* Per-particle signatures (Sec. 3.5): 16 TEA rounds on (bit-reversed tag,
 * the leading 11 mantissa bits of v_x, v_y, v_z interleaved, x lowest, the
 * 33rd bit dropped), keys (seed low, seed high, step low, step high), the
 * two halves xor-ed.  v: device double[3][n]; sig: device uint32[n]. */
int dpd_tea_signatures(int32_t n, const uint32_t* tag, const double* v, uint64_t step, uint64_t seed,
                       uint32_t* sig, void* stream);

/* Pair Gaussians from signatures: 4 TEA rounds on (min, max) of the two
 * signatures (same keys) give words (w0, w1); xi = sqrt(-2 ln u1)
 * cos(2 pi u2) with u1 = (w0 + 1/2) 2^-32, u2 = w1 2^-32, evaluated with
 * DPD_FN_FASTLOG and DPD_FN_FASTCOS2PI.  words (nullable): uint32[2 n]. */
int dpd_tea_gaussians(int64_t n, const uint32_t* sig_i, const uint32_t* sig_j, uint64_t step, uint64_t seed,
                      uint32_t* words, double* xi, void* stream);

/* Throughput probe: every thread t < n_tags draws the Gaussians of pairs
 * (t, t + 1), ..., (t, t + pairs_per_thread) (tags mod n_tags) and writes
 * their sum to sink[t].  generator 0: Philox4x32-10 and the device
 * library's log, sqrt and cospi (the FP64 force pass's generator);
 * generator 1: TEA-4 on sig[] (from dpd_tea_signatures) with the fast
 * logarithm and cosine.  pairs_per_thread < n_tags (else DPD_EINVAL). */
int dpd_gaussian_throughput(int32_t generator, int32_t n_tags, int32_t pairs_per_thread, uint64_t step,
                            uint64_t seed, const uint32_t* sig, double* sink, void* stream);

/* ---------------------------------------------------------------------------
 * Batched replicas
 *
 * Many independent periodic systems advanced together.  The paper hides
 * kernel-launch latency behind CUDA streams (Sec. 3.2.1); here every phase of
 * a step covers all systems in one launch (the particles, cells and 2x2x2
 * list blocks of all systems are numbered one after another), and a step
 * can be replayed as one HIP graph.
 *
 * A batch is described once by dpd_batch_create: per-system parameters and
 * particle ranges.  Systems may differ in box, particle count, a / gamma /
 * sigma tables, seed and body force; they share r_c, skin, dt, lambda, s and
 * n_types (the integrator and the weight form), and carry no bonds.  Within
 * system s, particles occupy [sys_offset[s], sys_offset[s+1]) of the
 * concatenated state and keep that range under reordering; tags are local
 * (a permutation of 0 .. n_s - 1 within each system), so the pair Gaussian of
 * a system equals that of the same system run alone.  Every system's
 * trajectory is bitwise equal to its single-system dpd_step run; per-system
 * statistics are summed in a different (fixed) order than dpd_step's.
 *
 * The handle is HOST memory allocated by dpd_batch_create and released by
 * dpd_batch_destroy; its device tables live in caller memory (d_table),
 * which must outlive the handle.  A handle may be used from one host thread
 * at a time.
 * ------------------------------------------------------------------------- */

typedef struct dpd_batch dpd_batch;

/* Launch shapes of the batched phases; any valid choice gives bitwise the
 * same results (only the speed differs). */
typedef struct dpd_tiles {
    int32_t force_grid;     /* workgroups of the persistent force pass,
                               64 .. 8192 (0 = one per 4 chunks of 64 rows,
                               at most 2048)                                   */
    int32_t nlist_waves;    /* waves per workgroup of the block and lane list
                               builders: 1, 2 or 4 (0 = 4); the tile builder
                               sizes its workgroups from the density          */
    int32_t nlist_kind;     /* list builder: 0 = one workgroup per 8x4x4-cell
                               tile with its neighbourhood staged in LDS,
                               2 = one lane per particle over global memory
                               (0 and 2 while the batch has fewer than 2^27
                               cells, else the block builder), 1 = one wave
                               per 2x2x2 cell block                            */
    int32_t reserved;       /* 0                                              */
} dpd_tiles;

/* Device bytes of the batch table for n_sys systems and n_total particles
 * (0 on invalid sizes). */
size_t dpd_batch_table_bytes(int32_t n_sys, int64_t n_total);

/* Describes a batch.  per_sys: host dpd_params[n_sys] (bond_partner must be
 * NULL); sys_offset: host int64[n_sys + 1], sys_offset[0] = 0, strictly
 * increasing, total below 2^31; n_sys in [1, 65535].  d_table: device memory
 * of dpd_batch_table_bytes(n_sys, total) bytes, 256-byte aligned; it is
 * filled by copies and one kernel enqueued on `stream`.  *out receives the
 * handle.  DPD_EINVAL for invalid parameters (the message names the
 * system), DPD_EUNSUPPORTED for bonds or for systems that differ in a
 * shared field, DPD_ECAPACITY for a short table. */
int dpd_batch_create(const dpd_params* per_sys, int32_t n_sys, const int64_t* sys_offset, void* d_table,
                     size_t table_bytes, void* stream, dpd_batch** out);

/* Releases the handle and its cached HIP graph (NULL is a no-op).  The
 * caller synchronises first if graph replays may still run. */
void dpd_batch_destroy(dpd_batch* b);

/* Totals of the concatenated arrays: particles and cells (cell_start of a
 * batch has n_cells_total + 1 entries).  Either pointer may be NULL. */
int dpd_batch_sizes(const dpd_batch* b, int64_t* n_total, int64_t* n_cells_total);

/* Workspace bytes for the batched calls in `precision` (0 on error). */
size_t dpd_batch_workspace_bytes(const dpd_batch* b, int32_t precision);

/* Launch shapes used by later calls (validated; DPD_EINVAL if out of range).
 * Changing them drops a cached graph. */
int dpd_batch_set_tiles(dpd_batch* b, const dpd_tiles* t);
int dpd_batch_get_tiles(const dpd_batch* b, dpd_tiles* t);

/* dpd_bin_reorder over all systems: each system's particles are binned in
 * its own box and reordered within its own range; cells are numbered
 * system by system, each system's in ascending Morton rank.  perm and
 * idx_of_tag hold batch-wide indices (idx_of_tag[sys_offset[s] + tag]). */
int dpd_batch_bin_reorder(const dpd_batch* b, const dpd_state* in, dpd_state* out, dpd_cells* cells,
                          float* x32, float* v32, void* ws, size_t ws_bytes, void* stream);

/* dpd_build_neighbors over all systems; list entries are batch-wide
 * indices and never cross a system. */
int dpd_batch_build_neighbors(const dpd_batch* b, const dpd_state* sorted, const dpd_cells* cells,
                              const float* x32, dpd_nlist* nl, int32_t* d_status, void* ws,
                              size_t ws_bytes, void* stream);

/* dpd_forces over all systems at `step`; pe_out (nullable, device
 * double[n_total]) gets each particle's share of the pair potential. */
int dpd_batch_forces(const dpd_batch* b, int32_t precision, const dpd_state* sorted, const dpd_cells* cells,
                     const float* x32, const float* v32, const dpd_nlist* nl, uint64_t step,
                     double* f_out, double* pe_out, int32_t* d_status, void* ws, size_t ws_bytes,
                     void* stream);

/* dpd_step over all systems (same preconditions per system, shared step
 * counter *d_step; the lists are rebuilt every step whatever the skin).  d_reductions (nullable): device double[n_steps][n_sys][8]
 * with dpd_step's eight per-step totals for every system.  use_graph != 0:
 * one step is captured into a HIP graph held by the handle (captured again
 * when an argument or the tiles change) and the graph is launched n_steps
 * times on `stream`; the results equal those of use_graph = 0.  As in
 * dpd_step, the steps' forces read each step's rows from the workspace and
 * nl's CSR index is written once, for the last step. */
int dpd_batch_step(dpd_batch* b, int32_t precision, dpd_state* st, int32_t n_steps, uint64_t* d_step,
                   double* d_reductions, dpd_cells* cells, dpd_nlist* nl, float* x32, float* v32,
                   int32_t* d_status, int32_t use_graph, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DPD_H */
