/*
 * lbm.h -- C ABI of the MI355X (gfx950) D3Q19 BGK lattice Boltzmann hot path.
 *
 * Method: Habich et al., "Performance engineering for the Lattice Boltzmann
 * method on GPGPUs" (Sec. 2, Eq. (1)): the BGK evolution equation on the
 * D3Q19 lattice with the equilibrium of Qian et al. (1992), updated with the
 * fused stream-collide ("pull") ordering and two lattices of Sec. 6; obstacle
 * cells handled by bounce-back (Sec. 2, last paragraph) in its half-way form;
 * body force by Guo, Zheng & Shi (Phys. Rev. E 65, 046308, 2002).  Options:
 * walls moving with one common velocity (the lid of the lid-driven cavity
 * the paper verifies on, Sec. 7), by Ladd's momentum-corrected bounce-back
 * (J. Fluid Mech. 271, 285, 1994) with reference density 1; and the
 * incompressible equilibrium of He & Luo (J. Stat. Phys. 88, 927, 1997) in
 * place of Qian's (the paper's "incompressible flow solver", abstract and
 * Sec. 2).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Lattice units (dx = dt = 1), c_s^2 = 1/3, nu = (tau - 1/2)/3.
 *  - Direction order i = 0..18 of every population array:
 *       0:( 0, 0, 0)  1:(+1, 0, 0)  2:(-1, 0, 0)  3:( 0,+1, 0)  4:( 0,-1, 0)
 *       5:( 0, 0,+1)  6:( 0, 0,-1)  7:(+1,+1, 0)  8:(-1,-1, 0)  9:(+1,-1, 0)
 *      10:(-1,+1, 0) 11:(+1, 0,+1) 12:(-1, 0,-1) 13:(+1, 0,-1) 14:(-1, 0,+1)
 *      15:( 0,+1,+1) 16:( 0,-1,-1) 17:( 0,+1,-1) 18:( 0,-1,+1)
 *    weights 1/3 (i = 0), 1/18 (i = 1..6), 1/36 (i = 7..18); opposite pairs
 *    (1,2) (3,4) (5,6) (7,8) (9,10) (11,12) (13,14) (15,16) (17,18).
 *  - Population grid ("grid"): structure of arrays [19][nz][ny][x_stride],
 *    x contiguous, x_stride >= nx from lbm_query (padding cells after each
 *    x-row, never computed -- the paper's Sec. 6 alignment padding); the 19
 *    direction arrays start dir_stride elements apart (dir_stride = nz * ny *
 *    x_stride + 256 bytes of padding, which keeps the arrays off power-of-two
 *    distances from each other), so element (i, z, y, x) is at
 *    i * dir_stride + (z * ny + y) * x_stride + x.  Each
 *    element of a fluid cell holds the OFFSET g_i = f_i - w_i of the
 *    post-collision population f*_i after the latest step, in the storage
 *    type:
 *      LBM_F32  float,  LBM_F64 double,  LBM_BF16 bfloat16 (g),
 *      LBM_F16  IEEE binary16 holding 2^s * g, s = f16_scale_log2.
 *    Every store rounds to nearest-even.  Collision arithmetic is FP32 for
 *    F32/F16/BF16 storage and FP64 for F64 and F32X storage.
 *    Solid cells carry no state of their own: every slot of a solid cell
 *    holds a marker (rewritten each step by the cell's own thread), one of
 *    two fixed quiet-NaN bit patterns of the storage type (LBM_MARK_* below,
 *    also returned by lbm_solid_markers): the moving-wall marker for a
 *    moving-wall cell when the wall velocity is not zero, else the resting
 *    one.  A pull whose raw bits equal a marker takes the half-way
 *    bounce-back value from the pulling cell's own opposite slot instead,
 *    plus the moving-wall term 6 w_i (c_i . u_w) in storage units for the
 *    moving-wall marker.  Any other value is data: a NaN or infinity that
 *    arises in a fluid cell (a 16-bit overflow, corrupted input) enters the
 *    neighbours' collisions and so reaches lbm_reduce as a non-finite sum.
 *    (The two-step pass at resting walls decides the same bounce-backs
 *    from a link mask built from the flags instead, with the same results.)
 *    Padding stays 0.  The library maintains the markers itself (init, step,
 *    save/restore); after writing a grid from outside, call
 *    lbm_refresh_solids.  Fluid values must never carry a marker pattern.
 *  - Scalar fields are [nz][ny][nx], vector fields [3][nz][ny][nx] (no
 *    padding).  flags are uint8 [nz][ny][nx]: bit0 LBM_FLAG_SOLID (obstacle
 *    cell, never read or written), bit1 LBM_FLAG_NOFORCE (fluid cell without
 *    body force), bit2 LBM_FLAG_MOVING (with bit0: a wall cell moving with
 *    lbm_params.wall_u; ignored without bit0); other bits are reserved and
 *    ignored.  flags == NULL means all fluid.
 *  - All axes are periodic; walls are rows of solid cells.
 *  - Time levels: after lbm_init the current grid holds f*(0) = f^eq(rho0,u0)
 *    (solid cells 0); each step streams with half-way bounce-back and then
 *    collides:  f*_i(x, t+1) = Omega_i( f_i(x, t+1) ),
 *      f_i(x, t+1) = f*_i(x - c_i, t)  if x - c_i is fluid, else f*_{opp i}(x, t)
 *                    (+ 6 w_i (c_i . u_w) if x - c_i is a moving wall).
 *  - Velocity: u = (j + F/2)/rho with Qian's equilibrium, u = j + F/2 with
 *    the incompressible one (rho0 = 1), j = sum f_i c_i.
 *  - Every pointer is device memory owned by the caller, 256-byte aligned,
 *    and must stay valid while work that uses it is queued.  Calls enqueue
 *    on the context's stream and return without synchronising; nothing in
 *    this library allocates device memory (the optional step graphs of
 *    lbm_use_graphs are the HIP runtime's).
 *  - Errors: every call returns lbm_status; LBM_OK = 0.  Invalid arguments
 *    are detected on the host before anything is enqueued (LBM_E_ARG) and
 *    leave the context unchanged.  lbm_last_error() gives a message for the
 *    calling thread's latest failure.  No C++ exception crosses this ABI.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Only the declarations below are exported from the shared library. */
#pragma GCC visibility push(default)

typedef enum {
  LBM_OK = 0,
  LBM_E_ARG = -1,         /* invalid argument (host-side validation) */
  LBM_E_HIP = -2,         /* a HIP runtime call or kernel launch failed */
  LBM_E_UNSUPPORTED = -3, /* valid but not supported (e.g. too large) */
  LBM_E_STATE = -4        /* call not valid for this context's state */
} lbm_status;

typedef enum {
  LBM_F32 = 0,  /* float offsets, FP32 collision arithmetic */
  LBM_F16 = 1,  /* binary16 holding 2^s offsets, FP32 arithmetic */
  LBM_BF16 = 2, /* bfloat16 offsets, FP32 arithmetic */
  LBM_F64 = 3,  /* double offsets, FP64 arithmetic */
  LBM_F32X = 4  /* float offsets (same layout and bytes as LBM_F32), FP64
                   collision arithmetic: removes the arithmetic rounding
                   altogether (LBM_F32 already carries its momentum terms
                   compensated, so both reach the FP32 storage floor on slow
                   flows; F32X is about 3x closer on fast ones) */
} lbm_storage;

typedef enum {
  LBM_EQ_QIAN = 0,           /* f^eq_i = w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u] */
  LBM_EQ_INCOMPRESSIBLE = 1  /* f^eq_i = w_i [rho + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u] */
} lbm_equilibrium;

enum { LBM_FLAG_SOLID = 1, LBM_FLAG_NOFORCE = 2, LBM_FLAG_MOVING = 4 };

/* Solid-cell markers: raw bits of a stored element (sign set, quiet NaN,
 * fixed payload; the moving-wall marker is the resting one with bit 0 set). */
#define LBM_MARK_F32_REST 0xFFD0D0D0u /* LBM_F32 and LBM_F32X */
#define LBM_MARK_F32_MOVING 0xFFD0D0D1u
#define LBM_MARK_F64_REST 0xFFFD0D0D0D0D0D0Cull
#define LBM_MARK_F64_MOVING 0xFFFD0D0D0D0D0D0Dull
#define LBM_MARK_F16_REST 0xFED4u
#define LBM_MARK_F16_MOVING 0xFED5u
#define LBM_MARK_BF16_REST 0xFFD4u
#define LBM_MARK_BF16_MOVING 0xFFD5u

/* lbm_params.steps_per_pass value for the automatic choice between one and
 * two steps per kernel pass. */
#define LBM_STEPS_AUTO (-1)

typedef struct {
  int32_t nx, ny, nz;     /* cells per axis, each >= 1 */
  int32_t storage;        /* lbm_storage */
  int32_t f16_scale_log2; /* s in [-24, 24]; used by LBM_F16 only */
  int32_t x_align;        /* x_stride is rounded up to a multiple of this many
                             cells; 0 = default (64), 1 = no padding */
  double tau;             /* BGK relaxation time, > 1/2, or +INFINITY
                             (omega = 0: pure streaming, a test mode) */
  double force[3];        /* Guo body-force density, finite */
  double wall_u[3];       /* velocity of the cells flagged SOLID | MOVING,
                             finite (tangential to the wall for a physical
                             moving wall); all 0 = every wall at rest */
  int32_t equilibrium;    /* lbm_equilibrium */
  int32_t obstacle_kernel; /* 0: bounce-back fused into the pull through the
                              solid markers (default); 1: the paper's split
                              design (Sec. 7), a separate kernel writing the
                              bounce-back values into the solid cells' slots
                              of the source grid before each step (for the
                              measured comparison; with it lbm_step_from
                              rewrites the solid-cell slots of src) */
  int32_t steps_per_pass; /* 0 or 1: one step per kernel pass; 2: lbm_step
                             runs pairs of steps as one fused pass that keeps
                             the intermediate level on chip (temporal
                             blocking along z, half the HBM traffic of two
                             passes), bit-identical to single steps; an odd
                             remainder is one single step.  Not with
                             obstacle_kernel = 1 (LBM_E_UNSUPPORTED).
                             LBM_STEPS_AUTO: pairs where the fused pass fills
                             the GPU (at least 128 blocks of its tiles: from
                             about 128^3 cells on), single steps elsewhere and
                             with the split design -- the fastest schedule
                             measured, the same bits either way. */
} lbm_params;

typedef struct lbm_ctx lbm_ctx;

/* Sizes the caller must allocate for `p` (any output pointer may be NULL).
 * The layout is the structure of arrays of Sec. 6 (one array per direction,
 * x fastest) with each row padded as Sec. 6 pads for aligned access, here to
 * x_align cells:
 *   x_stride       padded x extent of a grid row, in cells;
 *   dir_stride     elements from one direction array to the next;
 *   grid_bytes     bytes of ONE population grid (two are needed);
 *   scratch_bytes  bytes of the scratch passed to lbm_init: the reduction's
 *                  partials and, when steps_per_pass is 2 or LBM_STEPS_AUTO
 *                  (and two direction arrays span less than 4 GiB), 4 bytes
 *                  per cell for the two-step pass's link mask;
 *   adj_partials_bytes  bytes of the dL/dF partial-sum buffer of the adjoint.
 * Errors: LBM_E_ARG for invalid parameters, LBM_E_UNSUPPORTED when one
 * direction's array would exceed 4 GiB - 1 or a grid exceeds 2^31 cells. */
lbm_status lbm_query(const lbm_params* p, int64_t* x_stride, int64_t* dir_stride,
                     size_t* grid_bytes, size_t* scratch_bytes, size_t* adj_partials_bytes);

/* Algorithmic HBM bytes of one fluid-cell update for a storage type: 19 loads
 * + 19 stores of one population (Sec. 4 byte model: 152 for FP32, 304 for
 * FP64; 76 for the 16-bit offset storage).  Returns 0 for an unknown type. */
int32_t lbm_bytes_per_update(int32_t storage);

/* Copies the D3Q19 tables in the interface order above: e[19][3], w[19],
 * opp[19] (any pointer may be NULL).  Host memory; needs no GPU.  The set
 * is the 19-velocity lattice of Sec. 2 with the weights of Qian et al.
 * (1992), which the paper's equilibrium defers to. */
void lbm_lattice(int32_t* e, double* w, int32_t* opp);

/* Raw bits of the resting and the moving-wall solid marker of a storage
 * type (the LBM_MARK_* values; zero-extended for 16- and 32-bit types).
 * Host only.  Errors: LBM_E_ARG for an unknown storage type or a NULL
 * output. */
lbm_status lbm_solid_markers(int32_t storage, uint64_t* rest, uint64_t* moving);

/* Creates a context over caller-owned memory and enqueues the initial state
 * f*(0) = f^eq(rho0, u0) (Sec. 2 step 2 equilibrium) on fluid cells of
 * grid_a, the solid markers on its solid cells; everything else of both
 * grids (padding included) is set to 0.
 *   grid_a, grid_b  two grids of grid_bytes (the two lattices of Sec. 2);
 *   flags           uint8 [nz][ny][nx] or NULL (all fluid);
 *   scratch         scratch_bytes of device memory (lbm_reduce's partials;
 *                   with flags and resting walls, the link mask that the
 *                   two-step pass reads -- bit i of a cell set when its pull
 *                   along c_i comes from a solid cell, built here from the
 *                   flags);
 *   rho0            float [nz][ny][nx] or NULL (uniform 1);
 *   u0              float [3][nz][ny][nx] or NULL (rest);
 *   stream          a hipStream_t (NULL = default stream).
 * flags, scratch and the grids must outlive the context.  *out receives the
 * context (host memory, freed by lbm_destroy).
 * Errors: LBM_E_ARG (NULL out/p/grids/scratch, misaligned pointers, bad
 * params), LBM_E_UNSUPPORTED (size limits), LBM_E_HIP (launch failure). */
lbm_status lbm_init(lbm_ctx** out, const lbm_params* p, void* grid_a, void* grid_b,
                    const uint8_t* flags, void* scratch, const float* rho0,
                    const float* u0, void* stream);

/* Enqueues n >= 0 fused stream-collide steps (pull streaming with half-way
 * bounce-back, moments, equilibrium, BGK relaxation with Guo forcing: Sec. 2
 * steps 1-3, Eq. (1)), alternating between the two grids (each kernel pass
 * writes the other grid: one step, or two with steps_per_pass = 2).
 * Errors: LBM_E_ARG (NULL ctx, n < 0), LBM_E_HIP (launch failure). */
lbm_status lbm_step(lbm_ctx* ctx, int32_t n);

/* One step from an arbitrary grid `src` (state f*(t), same layout) into
 * `dst` (receives f*(t+1)); the context's own grids and time are untouched.
 * src and dst must differ.  Used to recompute forward states for the adjoint.
 * With obstacle_kernel = 1 the solid-cell slots of src (which carry no state)
 * are rewritten; its fluid values are not.  Errors: LBM_E_ARG, LBM_E_HIP. */
lbm_status lbm_step_from(lbm_ctx* ctx, const void* src, void* dst);

/* Two steps from an arbitrary grid `src` (state f*(t)) in one fused pass
 * (the steps of lbm_step_from twice, bit for bit): `mid` receives f*(t+1)
 * and `dst` f*(t+2); the context's own grids and time are untouched.  src,
 * mid and dst must be distinct, 256-byte aligned grids of the context's
 * layout.  Used by the adjoint's recomputation of the forward states
 * between checkpoints (one read of f* per two states).  Errors: LBM_E_ARG,
 * LBM_E_UNSUPPORTED (storage other than LBM_F32, or obstacle_kernel = 1),
 * LBM_E_HIP. */
lbm_status lbm_step2_from(lbm_ctx* ctx, const void* src, void* mid, void* dst);

/* Macroscopic fields of the current time level t from the stored f*(t):
 * the moments of Sec. 2 (density and momentum as the zeroth and first
 * moments of the populations, the quantities of the collision step),
 * rho = sum f*_i, rho u = sum f*_i c_i - F/2 (equal to the pre-collision
 * moments of step t under Guo forcing; F = 0 on no-force cells; rho0 u with
 * rho0 = 1 for the incompressible equilibrium).  Solid
 * cells get rho = 0, u = 0.  Either output may be NULL.  The _f64 variant
 * computes and writes in FP64.  Errors: LBM_E_ARG, LBM_E_HIP. */
lbm_status lbm_macroscopics(lbm_ctx* ctx, float* rho, float* u);
lbm_status lbm_macroscopics_f64(lbm_ctx* ctx, double* rho, double* u);

/* Global FP64 sums over fluid cells of the current time level:
 * out5 = {sum rho, sum rho u_x, sum rho u_y, sum rho u_z, sum rho |u|^2 / 2}
 * (rho0 = 1 in place of rho in the last four for the incompressible
 * equilibrium),
 * written to DEVICE memory out5 (5 doubles).  Deterministic (fixed-order
 * two-pass tree reduction, no atomics); uses the context's scratch.
 * Errors: LBM_E_ARG, LBM_E_HIP. */
lbm_status lbm_reduce(lbm_ctx* ctx, double* out5);

/* lbm_reduce without the context's scratch, for callers that cannot
 * allocate device memory or hand over a workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and result, bit for bit, with the partial sums in a static device
 * array of the library -- 1024 records of 5 doubles (40 KiB) per GPU, held
 * from the first lbm_init on that GPU until the process ends.  The
 * reduction uses exactly that many records for any grid size, so no grid is
 * too large.  It allocates nothing and does not synchronise.  Every call on
 * one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (other streams, other threads, other contexts) race and must be ordered
 * by the caller.  Errors: LBM_E_ARG, LBM_E_HIP. */
lbm_status lbm_reduce_noalloc(lbm_ctx* ctx, double* out5);

/* Context state: which grid (0 = grid_a, 1 = grid_b) holds f*(t), the step
 * count t, and the stream.  lbm_set_current declares that grid `parity`
 * holds f*(t) (for restoring a saved state). */
int32_t lbm_current(const lbm_ctx* ctx);
int64_t lbm_time(const lbm_ctx* ctx);
lbm_status lbm_set_current(lbm_ctx* ctx, int32_t parity, int64_t t);
lbm_status lbm_set_stream(lbm_ctx* ctx, void* stream);

/* Rewrites the solid markers of the current grid (needed only after the
 * caller has written populations into a grid directly) and the link mask
 * from the flags (needed after the caller has changed the flags).  No-op
 * without flags.  Errors: LBM_E_ARG, LBM_E_HIP. */
lbm_status lbm_refresh_solids(lbm_ctx* ctx);

/* Device-to-device copy of the current grid to `dst` (lbm_save), or of `src`
 * into the current grid with time t (lbm_restore); grid_bytes each, enqueued
 * on the context's stream.  Checkpoint / resume.  Errors: LBM_E_ARG, LBM_E_HIP. */
lbm_status lbm_save(lbm_ctx* ctx, void* dst);
lbm_status lbm_restore(lbm_ctx* ctx, const void* src, int64_t t);

/* ---- discrete adjoint (LBM_F32 / LBM_F32X storage) ------------------------
 * Reverse mode of the update above for an objective L of the final
 * macroscopic fields (FP32 adjoint arithmetic), with either equilibrium and
 * with moving walls (the wall velocity is a constant of the map, so it
 * enters the recomputed state but not the transpose; no gradient is formed
 * for it).  The carried adjoint state is nu^n = dL/df(n), the adjoint of
 * the PRE-collision populations f(n) = P f*(n-1) (P: the pull streaming with
 * half-way bounce-back); with lambda^n = dL/df*(n) = P^T nu^{n+1},
 *   nu^n = J(f(n))^T lambda^n,   dL/dF += JF(f(n))^T lambda^n,
 * J and JF the collision's Jacobians with respect to f and the force.  Each
 * call gathers what it needs (P^T as a pull along +c_i, P along -c_i) and
 * stores nu at the cell itself, so every store is aligned.  nu grids are
 * FP32 in the grid layout (grid_bytes of floats, direction arrays
 * dir_stride apart); the kernels write every cell of them, the resting solid
 * marker on solid cells, and never the padding.  dL/dF is accumulated per
 * thread block in an FP64 partials buffer (adj_partials_bytes) without
 * atomics; lbm_adjoint_finish_dF reduces it in a fixed order.  A rollout of
 * T steps: seed with f*(T-1); step with f*(n-1) for n = T-1 .. 1; init.
 * Errors: LBM_E_UNSUPPORTED for other storage types, LBM_E_ARG, LBM_E_HIP. */

/* Seed: nu^T = J(f(T))^T lambda^T, f(T) = P f*(T-1) gathered from fstar_prev
 * (= f*(T-1), grid layout), with lambda^T from dL/drho_T (float [nz][ny][nx]
 * or NULL = 0) and dL/du_T (float [3][nz][ny][nx] or NULL = 0):
 *   lambda^T_i = dL/drho + dL/du . (c_i - u)/rho
 * (dL/drho + dL/du . c_i for the incompressible equilibrium), where rho and
 * u are the moments of f(T) -- equal to the fields lbm_macroscopics reads
 * from f*(T).  (Re)initialises the partials with -dL/du / (2 rho) + JF^T
 * lambda^T (rho -> 1 for the incompressible equilibrium). */
lbm_status lbm_adjoint_seed(lbm_ctx* ctx, const void* fstar_prev, const float* dL_drho,
                            const float* dL_du, float* nu_T, double* dLdF_partials);

/* One reverse step n+1 -> n: lambda^n_i(x) = nu^{n+1}_i(x + c_i), or
 * nu^{n+1}_{opp i}(x) if x + c_i is solid; f(n) = P fstar_prev with
 * fstar_prev = f*(n-1); nu_n <- J(f(n))^T lambda^n; partials += JF^T
 * lambda^n.  nu_n must differ from both inputs. */
lbm_status lbm_adjoint_step(lbm_ctx* ctx, const void* fstar_prev, const float* nu_np1,
                            float* nu_n, double* dLdF_partials);

/* Initial-state adjoint from nu^1: lambda^0 = P^T nu^1 (gathered as above),
 * dL/du0 = sum_i lambda^0_i d f^eq_i/du (rho0, u0), written as float
 * [3][nz][ny][nx] (0 on solid cells).  rho0 / u0 as passed to lbm_init
 * (u0 NULL = rest, rho0 NULL = 1). */
lbm_status lbm_adjoint_init(lbm_ctx* ctx, const float* nu_1, const float* rho0,
                            const float* u0, float* dL_du0);

/* Fixed-order reduction of the partials into dLdF3 (3 doubles, device). */
lbm_status lbm_adjoint_finish_dF(lbm_ctx* ctx, const double* dLdF_partials, double* dLdF3);

/* ---- measurement ---------------------------------------------------------
 * STREAM copy c = a (the paper's Sec. 3 case study) over n_bytes of device
 * memory on `stream`, for the attainable-bandwidth denominator.  Both
 * pointers 256-byte aligned, n_bytes a multiple of 16. */
lbm_status lbm_stream_copy(void* c, const void* a, size_t n_bytes, void* stream);

/* Variants of the copy for the attainable-bandwidth sweep (the paper finds
 * the sustainable bandwidth by sweeping its STREAM copy over launch shapes,
 * Sec. 3): vec_per_thread in {1, 2, 4} 16-byte elements per thread per pass,
 * nontemporal = 1 for non-temporal loads and stores, blocks = the number of
 * 256-thread blocks striding through the array (0 or more than one pass
 * needs: exactly one pass).  Pointers and n_bytes as for lbm_stream_copy.
 * Errors: LBM_E_ARG, LBM_E_HIP. */
lbm_status lbm_copy_probe(void* c, const void* a, size_t n_bytes, int32_t vec_per_thread,
                          int32_t nontemporal, int32_t blocks, void* stream);

/* The same model with the access pattern of the step itself: one pure
 * streaming pass dst_i(x) = src_i(x - c_i) over the context's grid layout
 * (periodic in every axis; flags, walls and collision ignored), launched
 * exactly like the step kernel -- 19 shifted loads and 19 full-line stores
 * per cell.  Its rate is the bandwidth this memory pattern attains on the
 * device, the denominator that isolates the step's own overheads.  src and
 * dst are distinct grids of grid_bytes (256-byte aligned); the context's
 * grids and time level are untouched.  Errors: LBM_E_ARG, LBM_E_HIP. */
lbm_status lbm_pull_copy(lbm_ctx* ctx, const void* src, void* dst);

/* Launch-bound runs (small grids): with steps_per_graph = G (even, 2..4096)
 * lbm_step replays HIP graphs of G captured steps on the context's stream
 * and launches the remaining n mod G steps one by one; results are
 * bit-identical to plain launches.  This call captures the two graphs (one
 * per starting grid, on a library-owned stream; only the step kernels are
 * recorded) and instantiates them, so lbm_step itself only enqueues.  The
 * HIP runtime owns the graphs' resources.  Changing G (0 turns replays off,
 * the default) or destroying the context first waits on the host for the
 * latest replay -- through an event recorded after it, so also after
 * lbm_set_stream and after the caller destroyed the stream it ran on -- and
 * releases the old graphs.  Errors: LBM_E_ARG, LBM_E_HIP (graphs off). */
lbm_status lbm_use_graphs(lbm_ctx* ctx, int32_t steps_per_graph);

/* Destroys a context: its host memory and, if graphs were used, the graphs
 * (after waiting for their latest replay); device memory stays the caller's. */
void lbm_destroy(lbm_ctx* ctx);

/* Message of the calling thread's latest error ("" if none). */
const char* lbm_last_error(void);

#pragma GCC visibility pop

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
