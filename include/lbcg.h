/*
 * lbcg.h -- C ABI of the MI355X (gfx950) implementation of the improved
 * three-dimensional colour-gradient lattice Boltzmann model of Wen, Li, Yu &
 * Luo (arXiv 1904.03618): two immiscible fluids, red (k = 0) and blue (k = 1),
 * each carried by a D3Q19 distribution (Eq. 1, 5), advanced by the MRT
 * collision with the improved equilibrium and the error-cancelling correction
 * term (Eq. 18, 40-49), the tau-independent perturbation (Eq. 8, 53), the
 * Latva-Kokko recoloring (Eq. 10-12) and streaming (text after Eq. 12) with
 * periodic, halfway bounce-back and wetting walls.
 *
 * Conventions shared by every call:
 *   - node order is x-fastest: node = x + nx*(y + ny*z);
 *   - every GPU operation is enqueued on the HIP stream given to lbcg_init
 *     (NULL = the legacy default stream); calls are asynchronous except
 *     lbcg_moments (which returns FP64 sums to the host) and the periodic
 *     stability check inside lbcg_step;
 *   - one handle must not be used from two host threads at once;
 *   - every call returns LBCG_OK (0) or a negative error code; the text of the
 *     last error of the calling thread is available from lbcg_last_error().
 */
#ifndef LBCG_H
#define LBCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBCG_OK 0
#define LBCG_EINVAL (-1)     /* invalid argument (sizes, parameters, pointers) */
#define LBCG_ENOMEM (-2)     /* device allocation failed */
#define LBCG_EDEVICE (-3)    /* a HIP call failed */
#define LBCG_EUNSTABLE (-4)  /* NaN/Inf or negative colour density detected */
#define LBCG_ESTATE (-5)     /* NULL, freed or otherwise unusable handle */

#define LBCG_PERIODIC 0
#define LBCG_WALL 1          /* halfway bounce-back wall half a link beyond the
                                first and last node of the axis */

/* Population storage formats.  Every format stores each population as its
 * deviation from the rest state rho_k phi_i^k of the node that wrote it, next
 * to that node's FP32 colour densities (8 B per node); arithmetic is FP32. */
#define LBCG_FP32 0          /* FP32 deviations (152 B per node) */
#define LBCG_FP16S 1         /* FP16 deviations scaled by 2^10 (76 B per node) */
#define LBCG_BF16S 2         /* BF16 deviations (76 B per node) */

/*
 * One independent simulation box.  Fluid parameters follow the paper:
 *   rho_in    rho_R^in, rho_B^in, the reference densities of the phase field
 *             rho^N (text after Eq. 8); must satisfy the pressure balance
 *             rho_R^in (1 - alpha_R) = rho_B^in (1 - alpha_B) (Sec. IV.A)
 *             to 1e-12 relative;
 *   alpha     alpha_R, alpha_B of the pressure weights phi_i^k (Eq. 13), in [0, 1);
 *   tau_v     bulk shear relaxation times tau_v^R, tau_v^B (Eq. 52), > 1/2;
 *   A         surface-tension parameters A_R, A_B (Eq. 8); with the Eq. (53)
 *             form sigma = 2 (A_R + A_B) / 9;
 *   beta      recoloring parameter (Eq. 10-11);
 *   delta     half-width of the tau_v interpolation (Eq. 52, 0.98 usual);
 *   tau_e, tau_q, tau_pi   remaining relaxation times of S (Eq. 44), > 1/2;
 *   force     uniform body-force density (lattice units);
 *   grav, rho_ref          buoyancy: the force density at a node is
 *             force + (rho - rho_ref) * grav;
 *   bc        per axis LBCG_PERIODIC or LBCG_WALL; at most one axis may be a wall;
 *   theta_deg contact angle, measured through the red fluid, of the low and
 *             high wall of the wall axis (90 = neutral);
 *   improved  1: improved model (Eq. 18 equilibrium + correction term Eq. 45);
 *             0: the same MRT model without both improvements;
 *   meq4      rows 16-18 of the moment equilibria: 0 = M f^eq (the definition
 *             the text gives for m^eq, and the default), 1 = the rows as the
 *             Appendix prints them (2 rho_k c^2 (u_a^2 + u_b^2) in place of
 *             the 3 rho_k (u_a^2 + u_b^2) of M f^eq); other values LBCG_EINVAL;
 *   wall_u    velocity of the low and high wall of the wall axis (moving
 *             plates, Sec. IV.A); tangential only (the component along the
 *             wall axis must be 0) and zero when no axis is a wall.  A
 *             population reflected at a moving wall gains
 *             f_i^{k,eq}(rho_k, U_w) - f_opp(i)^{k,eq}(rho_k, U_w), twice the
 *             odd part of the case's equilibrium (Eq. 18, or Eq. 6 when
 *             improved = 0) at the wall velocity, rho_k the node's colour
 *             density; a uniform flow at U_w is then left unchanged.  Non-finite
 *             or non-tangential velocities give LBCG_EINVAL.
 */
typedef struct lbcg_case {
    int32_t nx, ny, nz;
    int32_t bc[3];
    double theta_deg[2];
    double rho_in[2];
    double alpha[2];
    double tau_v[2];
    double A[2];
    double beta, delta;
    double tau_e, tau_q, tau_pi;
    double force[3];
    double grav[3];
    double rho_ref;
    int32_t improved;
    int32_t meq4;
    double wall_u[2][3];
} lbcg_case;

/* Initial fields of one case: FP64 arrays of nx*ny*nz values, x-fastest.
 * on_device = 0: host memory; 1: device memory.  Read once during lbcg_init;
 * the caller keeps ownership. */
typedef struct lbcg_fields {
    const double *rhoR, *rhoB, *ux, *uy, *uz;
    int32_t on_device;
    int32_t reserved;
} lbcg_fields;

/* Step kernels. */
#define LBCG_KERNEL_AUTO 0      /* the fused step when every case allows it, else two-pass */
#define LBCG_KERNEL_TWOPASS 1   /* moments pass + collision pass (any boundaries) */
#define LBCG_KERNEL_FUSED 2     /* single pass, z-marching 32 x 8 tiles with the
                                   phase-field halo in LDS; eligible cases: no
                                   walls, or walls on the z axis (any contact
                                   angle, at rest or moving) */

/* Level formats (how a time level is stored between steps). */
#define LBCG_LEVEL_AUTO 0       /* FP32 with the fused step: compact; otherwise pairs */
#define LBCG_LEVEL_PAIR 1       /* every direction stores its red and blue deviation */
#define LBCG_LEVEL_COMPACT 2    /* fused step only: direction 0 stores both colours,
                                   directions 1-18 only the total deviation, and each
                                   node 7 FP32 words from which the reader rebuilds the
                                   red share exactly as the recoloring (Eq. 10-11)
                                   split it; 27 words per node and level in FP32
                                   instead of 40.  The start level and a level written
                                   by lbcg_set_fields are pairs; the first step
                                   after them writes the compact format. */

/* Handle-wide options.  storage: LBCG_FP32 / LBCG_FP16S / LBCG_BF16S.
 * diag_every: run the stability check every this many steps inside
 * lbcg_step (0 = never).  block_nodes: nodes per work tile and workgroup of
 * the two-pass kernels (0 = default 256; 64, 128, 192 or 256).
 * persistent_blocks: 0 = one workgroup per tile, >0 = that many workgroups
 * looping over all tiles of all cases (batched persistent launch).
 * kernel: LBCG_KERNEL_*.  zchunk: z-planes per fused tile (0 = default: with
 * T(zc) tiles of all cases and S workgroup slots for the fused kernel the
 * handle runs (CUs x the workgroups per CU that its registers and LDS allow,
 * queried from the runtime at init; a failed query is LBCG_EDEVICE), the
 * chunk in 8 .. 128 planes (FP32) or 8 .. 64 (16-bit forms) that minimises
 * ceil(T / S) (zc + 2), the longer on a tie, or the longest where that one
 * gives T >= 2 S; lbcg_zchunk reports it).
 * graph_steps: 0 = launch every kernel of every step; n > 0 = capture n steps
 * (rounded up to even) once into a HIP graph and replay it; with diag_every
 * the stability check then runs at the first replay boundary at or after each
 * multiple of diag_every, and kernel timing (lbcg_timing) is not available.
 * level: LBCG_LEVEL_*; LBCG_LEVEL_COMPACT with the two-pass step (asked for,
 * or the only one the cases allow) is LBCG_EINVAL. */
typedef struct lbcg_options {
    int32_t storage;
    int32_t diag_every;
    int32_t block_nodes;
    int32_t persistent_blocks;
    int32_t kernel;
    int32_t zchunk;
    int32_t graph_steps;
    int32_t level;
} lbcg_options;

typedef struct lbcg_handle lbcg_handle;

/*
 * Create a handle for n_cases independent boxes and set every case to the
 * equilibrium f^k = f^{k,eq}(rho_k, u0) of the improved (Eq. 18) or original
 * (Eq. 6) equilibrium at time level 0.  hip_stream is a hipStream_t (may be
 * NULL).  On success *out receives the handle, which owns all device memory
 * it allocates.  Errors: LBCG_EINVAL (n_cases < 1, any dimension < 1, more
 * than 2^28 - 64 nodes in one case (the kernels use 32-bit byte offsets within
 * a case; a larger domain is split into cases or GPUs), more than one wall
 * axis, alpha outside [0,1), a relaxation time <= 1/2, rho_in <= 0, broken
 * pressure balance, a non-tangential or non-finite wall velocity, NULL
 * pointer), LBCG_ENOMEM, LBCG_EDEVICE.
 */
int lbcg_init(const lbcg_case *cases, int32_t n_cases, const lbcg_fields *init,
              const lbcg_options *opt, void *hip_stream, lbcg_handle **out);

/*
 * Advance every case by nsteps time steps.  One step: moments (Eq. 4), phase
 * field and colour gradient (Eq. 8, 49), correction gradients (Eq. 46-49),
 * tau_v (Eq. 52), MRT collision with correction, force and perturbation in
 * moment space (Eq. 41-45, 53), recoloring (Eq. 10-11), pull streaming with
 * periodic wrap or halfway bounce-back.  Errors: LBCG_ESTATE, LBCG_EINVAL
 * (nsteps < 0), LBCG_EDEVICE, LBCG_EUNSTABLE (the stability check found a
 * NaN/Inf or a colour density below -1e-3 rho_in; lbcg_steps_done() then
 * tells the level that failed).
 */
int lbcg_step(lbcg_handle *h, int64_t nsteps);

/*
 * Macroscopic fields of case case_id at the current level (post-streaming,
 * before collision): rho_R, rho_B, the phase field rho^N and the mixture
 * velocity u = (sum_ik e_i f_i^k + F/2)/rho.  Each field pointer is caller-owned
 * DEVICE memory of nx*ny*nz FP32 values, or NULL to skip it.  diag, if not
 * NULL, is caller-owned HOST memory for 5 FP64 sums over the case:
 * {sum rho_R, sum rho_B, sum rho u_x, sum rho u_y, sum rho u_z}; the call then
 * synchronises the stream.  Errors: LBCG_ESTATE, LBCG_EINVAL (bad case_id),
 * LBCG_EDEVICE.
 */
int lbcg_moments(lbcg_handle *h, int32_t case_id, float *rhoR, float *rhoB, float *rhoN,
                 float *ux, float *uy, float *uz, double *diag);

/* Reset case case_id to the equilibrium f^k = f^{k,eq}(rho_k, u) of the given
 * fields (as lbcg_init does at level 0), keeping the handle's step count: the
 * entry through which predicted macroscopic fields re-enter the LB state.
 * fields: FP64 arrays as in lbcg_init.  Errors: LBCG_ESTATE, LBCG_EINVAL,
 * LBCG_ENOMEM, LBCG_EDEVICE. */
int lbcg_set_fields(lbcg_handle *h, int32_t case_id, const lbcg_fields *fields);

/* Release every device resource of the handle after the stream's pending work
 * has finished.  LBCG_ESTATE for NULL, for an already freed handle and for a
 * pointer lbcg_init never returned (the library keeps a registry of live
 * handles and never reads such a pointer).  Every other call also returns
 * LBCG_ESTATE (or -1) for such pointers. */
int lbcg_free(lbcg_handle *h);

/* ---- inspection helpers (tests, checkpoints) ---- */

/* Text of the calling thread's last error ("" if none). */
const char *lbcg_last_error(void);

/* Number of time steps the handle has completed. */
int64_t lbcg_steps_done(const lbcg_handle *h);

/* The streaming map the step kernels use: for every direction i and node,
 * src_node[i*N + node] and src_dir[i*N + node] name the post-collision value
 * that the pull at (node, i) reads.  Both are caller-owned DEVICE buffers of
 * 19*N entries.  Errors: LBCG_ESTATE, LBCG_EINVAL, LBCG_EDEVICE. */
int lbcg_index_map(lbcg_handle *h, int32_t case_id, int64_t *src_node, int8_t *src_dir);

/* Decoded FP32 populations of case case_id at the current level into
 * caller-owned DEVICE memory f[(k*19 + i)*N + node] (with compact levels the
 * red and blue shares are rebuilt from the writers' data exactly as the next
 * step rebuilds them).  Errors as above. */
int lbcg_get_populations(lbcg_handle *h, int32_t case_id, float *f);

/* Kernel timing with HIP events on the handle's stream.  enable = 1 starts
 * recording an event pair around every kernel of every following step
 * (enable = 0 stops).  lbcg_timing_read synchronises the stream and writes,
 * for the kernels {moments pass, wall ghost layer, collision pass, fused
 * step} (a handle on the fused step records only the last), the summed duration in milliseconds into ms[4] and the number of
 * recorded launches into launches[4]; it then clears the totals.  Errors: LBCG_ESTATE,
 * LBCG_EINVAL (NULL output), LBCG_EDEVICE. */
int lbcg_timing(lbcg_handle *h, int32_t enable);
int lbcg_timing_read(lbcg_handle *h, double *ms, int64_t *launches);

/* Number of nodes and storage bytes per population value of the handle;
 * the handle's step kernel (LBCG_KERNEL_TWOPASS or LBCG_KERNEL_FUSED), level
 * format (LBCG_LEVEL_PAIR or LBCG_LEVEL_COMPACT) and fused z-chunk in planes
 * (0 with the two-pass step) as resolved at init.  -1 for an invalid handle
 * or case. */
int64_t lbcg_case_nodes(const lbcg_handle *h, int32_t case_id);
int32_t lbcg_storage_bytes(const lbcg_handle *h);
int32_t lbcg_step_kernel(const lbcg_handle *h);
int32_t lbcg_level_format(const lbcg_handle *h);
int32_t lbcg_zchunk(const lbcg_handle *h);

/* Checkpoint / resume.  The state of a handle at its current level is the
 * stored population values of every case (raw bits, storage format of the
 * handle), the colour densities their writers stored with them (with compact
 * levels also the writers' recoloring data and, per case, whether its level
 * is still a pair-format start level), and the step count; everything else
 * (aux and ghost layers) is recomputed by the next step.  lbcg_checkpoint_bytes gives the size of that image (-1 for a
 * bad handle).  lbcg_checkpoint_save synchronises the handle's stream and
 * copies the image into caller-owned HOST memory of at least that size.
 * lbcg_checkpoint_load restores an image into a handle created with the same
 * case shapes, in the same case order, and storage format (the image records
 * every case's extents and array offsets and the load compares them;
 * parameters other than the shapes are the handle's own); the next steps then
 * continue bit for bit as the saved handle would have.  Errors: LBCG_ESTATE,
 * LBCG_EINVAL (NULL buffer, too small, or an image of other case extents,
 * case order, storage or level format), LBCG_EDEVICE. */
int64_t lbcg_checkpoint_bytes(const lbcg_handle *h);
int lbcg_checkpoint_save(lbcg_handle *h, void *host, int64_t bytes);
int lbcg_checkpoint_load(lbcg_handle *h, const void *host, int64_t bytes);

#ifdef __cplusplus
}
#endif

#endif /* LBCG_H */
