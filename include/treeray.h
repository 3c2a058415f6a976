/*
 * treeray.h -- C ABI of the MI355X (gfx950) TreeRay/RadPressure hot path.
 *
 * The library computes, for every cell of an AMR grid, the diffuse infrared radiation
 * field of Klepitko et al. (MNRAS 2023, "Tree-based solvers for adaptive mesh refinement
 * code FLASH - III"): every cell and every star particle is a source; rays from each
 * target cell are HEALPix pixels; octree nodes are mapped onto radial ray segments and
 * each ray is integrated in 1-D (Sec. 4).  Outputs are the fields the paper names:
 * mean intensity J (IRXE), flux F, radiation-pressure acceleration a_RP (RPAX/Y/Z),
 * trapped source pressure P_src (PRAD) and the dust temperature (TDUS) (Sec. 4).
 *
 * Conventions
 *  - All functions return an int status: TR_OK or a negative TR_E* code; the message of
 *    the last failure on a context is returned by tr_last_error().  No exception crosses
 *    the ABI.
 *  - "device" pointers are HIP device memory owned by the caller; the library never frees
 *    them.  "host" pointers are read during the call only.  Handles (tr_ctx, tr_tree,
 *    tr_mlp) are owned by the library and released by their *_free / *_destroy call.
 *  - Work is enqueued on the context's stream; calls return before the GPU finishes
 *    unless stated otherwise.  Device-side failures (stack overflow in the tree walk)
 *    are latched in the context and reported by tr_sync().
 *  - Cell arrays are block-major in the order of the grid's block list; inside a block of
 *    8^3 cells the cell (ci, cj, ck) has local offset ci + 8 cj + 64 ck.  Vector outputs
 *    are structure-of-arrays: F[0..n) = F_x, F[n..2n) = F_y, F[2n..3n) = F_z.
 *  - Units: cgs, or code units with sigma = pi and c = 1; the library uses only the
 *    sigma and c given in tr_units and the lengths given in tr_grid.
 */
#ifndef TREERAY_H
#define TREERAY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TR_OK = 0,
    TR_EINVAL = -1,    /* bad argument or grid (message says which) */
    TR_ENOMEM = -2,    /* device or host allocation failed */
    TR_EHIP = -3,      /* a HIP runtime call failed */
    TR_EOVERFLOW = -4, /* the walk's per-wave stack overflowed (results invalid) */
};

typedef struct tr_ctx tr_ctx;
typedef struct tr_tree tr_tree;
typedef struct tr_mlp tr_mlp;

/* AMR grid: a cubic domain of nb^3 base blocks, each leaf block of 8^3 cells at a
 * refinement level 0..max_level (level l has cell edge box_len / (8 nb 2^l)).
 * blocks is a HOST array [n_blk][4] = (level, bi, bj, bk), bi..bk in [0, nb 2^level).
 * Leaf blocks must tile the domain without overlap. */
typedef struct tr_grid {
    int32_t nb;
    int32_t max_level;
    int32_t n_blk;
    const int32_t *blocks;
    double x0[3];
    double box_len;
} tr_grid;

typedef struct tr_units {
    double sigma; /* Stefan-Boltzmann constant in the caller's units */
    double c;     /* speed of light */
} tr_units;

/* point source with non-ionising luminosity L_IR (Sec. 4.1.1); a host array for
 * tr_build_tree, a device array for tr_tree_refill */
typedef struct tr_star {
    double x, y, z, L;
} tr_star;

/* Tree build (Sec. 4.1 b-nodes; App. A h-nodes and centre of luminosity).
 * rho, t_dust: device float[n_cells]; kappa: device float[n_cells] or NULL, in which
 * case the Planck-mean dust opacity of t_dust is used (Sec. 2).  A cell is optically
 * thick when rho kappa dx >= 1.  The star host cell is the leaf containing (x, y, z)
 * with half-open cells.  Synchronises the stream once (to size the node arrays).
 * The tree keeps per-cell opacity and optical depth for tr_rad_force. */
int tr_build_tree(tr_ctx *ctx, const tr_grid *grid, const float *rho, const float *kappa,
                  const float *t_dust, const tr_star *stars, int n_stars,
                  const tr_units *units, tr_tree **out);
void tr_tree_free(tr_tree *tree);
/* Refill a tree's content for new cell fields and stars on the same blocks (Sec. 4.1.1 b-nodes,
 * App. A h-nodes and centres of luminosity): the same node arrays as tr_build_tree of the same
 * grid with these inputs, bit for bit, without allocating or synchronising, so it can be
 * captured in a graph with the calls that follow it.  rho, kappa (or NULL), t_dust as in
 * tr_build_tree; stars: DEVICE array of n_stars tr_star, 8-byte aligned (NULL when n_stars = 0).  The units
 * are the build's; no input validation.  Asynchronous. */
int tr_tree_refill(tr_ctx *ctx, tr_tree *tree, const float *rho, const float *kappa,
                   const float *t_dust, const tr_star *stars, int n_stars);

typedef struct tr_tree_info {
    int64_t n_node, n_leaf, n_cells;
    int32_t depth;     /* depth of the finest cells (root = 0) */
    int32_t root_edge; /* root edge in lattice units u = half the finest cell edge */
    int32_t n_bins;    /* ray evaluation points R_i = i^2 u, i = 1..n_bins */
    double u_len;      /* u in length units */
} tr_tree_info;
int tr_tree_get_info(const tr_tree *tree, tr_tree_info *info);

/* Copy the node arrays to HOST buffers (any may be NULL); synchronous.  Node order:
 * by depth, then Morton order of the node's integer coordinates; children of a node are
 * consecutive.  geo[n][4] = (centre x, y, z in u, first child or -1); meta[n] = depth |
 * child mask << 4 | leaf << 12 | (optically thick content) << 13; q[n][4] = leaf (L, A, S, 0) with the sign bit of L set
 * for optically thick leaves, h-node (L_thin, L_thick*V_thick, A_thin, A_thick);
 * vthick[n]; pcol[n][3] = mapping position in u/256; leaf_cell[n] = cell or -1.
 * Luminosities are in (length unit / u)^2 times the caller's units, areas in u^2. */
int tr_tree_export(tr_ctx *ctx, const tr_tree *tree, int32_t *geo, uint32_t *meta,
                   float *q, float *vthick, int32_t *pcol, int64_t *leaf_cell);

/* Ray tracing parameters (Sec. 4.2-4.4). */
typedef struct tr_trace_params {
    int32_t n_side;        /* HEALPix N_side: 1, 2, 4 or 8 (12 N_side^2 rays) */
    int32_t theta_num;     /* opening angle theta = num/den; 0/0 selects 1/(2 N_side) */
    int32_t theta_den;
    int32_t cube_m;        /* direction cells per cube-face edge of the angular kernel;
                              0 selects 16 N_side */
    int32_t merge;         /* 1: merge segments spanned by thick material (Sec. 4.3) */
    float j_bg;            /* background intensity entering at the ray ends */
    int32_t bins_per_pass; /* ray segments per walk pass (at most 16); 0 = automatic */
    int32_t chunk;         /* targets taken per work-queue grab; 0 = automatic */
    int32_t waves_per_block; /* waves per block; 0 = automatic */
    int32_t kernel;        /* 0 = automatic, 1 = one wave per target (segments processed in
                              passes of bins_per_pass radial points; the only kernel); 2 (one
                              block of waves per target) is withdrawn: TR_EINVAL */
    int32_t per_node_kernel; /* 0 = tabulated angular kernel (tr_alpha_table) for nodes at
                              least 8 edges away and the per-node 8-point kernel for nearer
                              ones; 1 = the per-node kernel for every node */
    int32_t orientation;   /* orientation of the ray set (Sec. 7.6): 0 = HEALPix axes, 1..47 =
                              a signed permutation of the axes applied to every target (axis
                              permutation o / 8 in the order 012 021 102 120 201 210, sign
                              flip of axis a for bit a of o % 8), -1 = one drawn per target
                              cell from SplitMix64(orient_seed * 2^32 + cell) mod 48 */
    uint32_t orient_seed;
    int32_t stack_limit;   /* test hook: ranges per wave walk stack; 0 = 56 depth + 8, which cannot
                              overflow.  A smaller value (at least 9) can: the walk then drops
                              subtrees, latches the overflow and tr_sync returns TR_EOVERFLOW */
} tr_trace_params;

/* Trace all cells of the tree: J (device float[n_cells], IRXE), F (device float[3][n],
 * flux), u_rad (device float[n_cells] = 4 pi J / c, or NULL).  Asynchronous; graph
 * capturable after the first call with the same N_side and cube_m (the first call builds
 * the angular-kernel table).  TR_EINVAL for a root edge above 2048 lattice units or a tree
 * of 2^28 nodes or more (limits of the walk's integer tests and record offsets). */
int tr_trace_rays(tr_ctx *ctx, const tr_tree *tree, const tr_trace_params *p, float *J,
                  float *F, float *u_rad);

/* Batched ray tracing: many trees (uneven AMR instances, each with its own N_side,
 * opening angle and outputs) traced by ONE persistent launch whose waves take targets
 * from the concatenated target lists; the launch is captured once in a HIP graph.
 * trees: HOST array [n] of tree handles; p: HOST array [n] of parameters (the knobs
 * bins_per_pass, chunk and waves_per_block of p[0] apply to the whole batch and are what
 * tr_batch_tune replaces); J, F, u_rad: HOST arrays [n] of device pointers (u_rad or its
 * entries may be NULL).  At most 4 distinct (N_side, cube_m) per batch.  The batch keeps
 * the pointers: trees and outputs must outlive it.  Creation synchronises the context's
 * stream. */
typedef struct tr_batch tr_batch;
int tr_batch_create(tr_ctx *ctx, int n, const tr_tree *const *trees, const tr_trace_params *p,
                    float *const *J, float *const *F, float *const *u_rad, tr_batch **out);
/* Replay the captured graph on the context's stream (asynchronous; no allocation). */
int tr_batch_launch(tr_batch *b);
/* The same work launched directly instead of through the graph (asynchronous). */
int tr_batch_launch_eager(tr_batch *b);
/* Autotuner: times the batch on every sample_stride-th target of each instance while
 * varying segments per pass, waves per block and the work-queue chunk (coordinate
 * descent), keeps the fastest and re-captures the graph.  Synchronous.  The outputs of
 * the sampled targets are overwritten. */
typedef struct tr_batch_tuning {
    int32_t bins_per_pass;   /* segments per pass; 0 = the longest pass each instance fits */
    int32_t waves_per_block; /* 0 = as many as the LDS holds */
    int32_t chunk;           /* targets per work-queue grab; 0 = 1 */
    float sample_ms;         /* output: time of the tuned launch on the sample (0 if not timed) */
    int32_t widest_pass;     /* output: most segments per pass of any instance under the setting */
    int32_t waves_used;      /* output: waves per block under the setting */
} tr_batch_tuning;
int tr_batch_tune(tr_batch *b, int sample_stride, tr_batch_tuning *best);
/* The batch's current setting (outputs filled as by tr_batch_tune). */
int tr_batch_get_tuning(const tr_batch *b, tr_batch_tuning *out);
/* Applies a setting, for instance one tr_batch_tune found in an earlier run and stored
 * (bins_per_pass, waves_per_block, chunk are read; the outputs are ignored), and
 * re-captures the graph, so that a cached tuning costs no new search.  TR_EINVAL for a
 * negative field or a setting that does not fit the LDS, in which case the batch keeps its
 * previous setting.  Synchronous. */
int tr_batch_set_tuning(tr_batch *b, const tr_batch_tuning *t);
void tr_batch_free(tr_batch *b);
/* One-shot batched trace (build descriptors, one persistent launch, free); synchronous. */
int tr_trace_rays_batched(tr_ctx *ctx, int n, const tr_tree *const *trees, const tr_trace_params *p,
                          float *const *J, float *const *F, float *const *u_rad);

/* Walk statistics of the opening-angle walk per target cell: counters (device
 * int32[n_cells][3] = b-nodes accepted, h-nodes accepted, h-nodes opened). */
int tr_walk_counts(tr_ctx *ctx, const tr_tree *tree, const tr_trace_params *p,
                   int32_t *counters);

/* Angular kernel table [6][M][M] (pixel id of each direction cell) and ray directions
 * [N_pix][3], built on the device and copied to HOST buffers; synchronous. */
int tr_ray_tables(tr_ctx *ctx, int n_side, int cube_m, int32_t *table, float *dirs);

/* Tabulated angular kernel (Sec. 4.2) that nodes at least 8 edges away use: HOST
 * int32[6 M M][15][9], per direction cell and distance class c = floor(log2(r^2 / s^2)) =
 * 6 .. 20, pixels 0..3 (ascending), their counts out of 64 sub-points, and a flag for keys
 * whose sub-points reach more than 4 pixels (served by the per-node kernel); synchronous. */
int tr_alpha_table(tr_ctx *ctx, int n_side, int cube_m, int32_t *out);

/* Radiation pressure (Sec. 4.5): a_RP = kappa F / c (1 - e^-tau)/tau with the factor 1
 * below tau = 1e-4, tau = rho kappa dx of the cell; P_src = (1 - e^{-tau/2}) L / (c dV^(2/3))
 * in cells hosting stars, 0 elsewhere.  F: device float[3][n]; a_rp: device
 * float[3][n]; p_src: device float[n] or NULL. */
int tr_rad_force(tr_ctx *ctx, const tr_tree *tree, const float *F, float *a_rp,
                 float *p_src);

/* Dust thermal equilibrium (Sec. 4.6, App. E).  Balance of thermal emission
 * xi 4 sigma rho kappa(T_d) T_d^4, absorption xi 4 pi rho kappa(T_J) J and gas-dust
 * collisional coupling c_gd n_H^2 sqrt(T_g) (T_g - T_d) (1 - 0.8 exp(-75/T_g)),
 * n_H = rho / (1.4 m_H); floor 2.7 K.  The root is unique and is found by Newton's
 * method inside a sign-changing bracket, falling back to bisection. */
typedef struct tr_dust_params {
    double sigma, c;
    double c_gd;      /* gas-dust coupling coefficient (erg s^-1 cm^3 K^-3/2) */
    double xi;        /* factor on the radiative rates (1 = kappa per gram of gas) */
    float rel_tol;    /* Newton stop |dT| <= rel_tol T (0 selects 1e-6) */
    int32_t max_iter; /* 0 selects 50 */
    int32_t start;    /* without a network: 0 = secant point of the bracket in (ln T, ln w),
                         1 = the bracket end with the smaller |ln(w/K)|, 2 = plain bisection
                         of the bracket (no Newton steps; a reference for the iteration
                         counts, stopping when the bracket width is <= rel_tol T) */
    int32_t linear;   /* 0 = Newton on ln w(T) against ln T, 1 = Newton on the residual g(T);
                         ignored by bisection */
    int32_t staged;   /* with a network: 0 = one kernel, the guesses kept in registers;
                         1 = the network's inference into a buffer, then the solve (the same
                         guesses and results; the form tr_dust_equilibrium_noalloc takes) */
} tr_dust_params;

/* rho, u_rad, t_gas: device float[n]; t_dust: device float[n]; iters: device uint8[n]
 * or NULL (Newton/bisection steps taken).  mlp: trained guess network (its output is the
 * starting point) or NULL for the plain start chosen by p->start.  With a network n must be
 * below 2^28. */
int tr_dust_equilibrium(tr_ctx *ctx, int64_t n, const float *rho, const float *u_rad,
                        const float *t_gas, const tr_dust_params *p, const tr_mlp *mlp,
                        float *t_dust, uint8_t *iters);

/* Allocation-free variant of tr_dust_equilibrium, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and results; with a network it always takes the staged form
 * (p->staged is ignored), whose starting temperatures go to a fixed scratch array of
 * TR_NOALLOC_DUST_STATES floats (16 MiB) that each
 * GPU holds from the library's first context on it until the process ends.  n above
 * TR_NOALLOC_DUST_STATES fails with TR_EINVAL before any work; the call makes no hipMalloc or
 * hipFree.  Every call on one GPU shares that GPU's array: calls that overlap in time on one
 * GPU (other streams or contexts) race, and the caller must order them.  Nothing in the array
 * has to start at zero: the network writes every starting point the solve then reads. */
#define TR_NOALLOC_DUST_STATES (1 << 22)
int tr_dust_equilibrium_noalloc(tr_ctx *ctx, int64_t n, const float *rho, const float *u_rad,
                                const float *t_gas, const tr_dust_params *p, const tr_mlp *mlp,
                                float *t_dust, uint8_t *iters);

/* Self-consistent dust temperature (Sec. 2, 4.1, 4.6): repeat tree build (Planck-mean
 * opacity and emission of the current T_dust; no kappa array), ray tracing and dust
 * equilibrium until the largest relative change of T_dust is <= tol or max_iter sweeps.
 * t_dust: device float[n], the starting temperature on entry and the result on return;
 * J, F, u_rad: device outputs of the last trace (as tr_trace_rays).  *iterations and
 * *max_rel_change (host, may be NULL) receive the sweeps done and the last change.
 * Synchronous (one readback per sweep). */
int tr_dust_fixed_point(tr_ctx *ctx, const tr_grid *grid, const float *rho, const float *t_gas,
                        const tr_star *stars, int n_stars, const tr_units *units,
                        const tr_trace_params *tp, const tr_dust_params *dp, const tr_mlp *mlp,
                        int max_iter, float tol, float *t_dust, float *J, float *F, float *u_rad,
                        int32_t *iterations, float *max_rel_change);

/* Guess network for the dust equilibrium: inputs (log10 rho, log10 u_rad, log10 T_gas)
 * normalised as (v - shift) * scale, output log10 T_d = y / out_scale + out_shift;
 * 3 -> 64 -> 64 -> 1 with ReLU hidden layers; BF16 MFMA with FP32 accumulation.
 * Parameters (HOST float, n = tr_mlp_n_params()) in the order
 * W1[64][3] b1[64] W2[64][64] b2[64] W3[64] b3. */
int tr_mlp_n_params(void);
int tr_mlp_create(tr_ctx *ctx, const float *params_host, const float *norm_host /* [8]:
                  shift[3], scale[3], out_shift, out_scale */, tr_mlp **out);
void tr_mlp_free(tr_mlp *mlp);
int tr_mlp_get_params(tr_ctx *ctx, const tr_mlp *mlp, float *params_host);
/* Training state, for checkpoint and resume: FP32 parameters, Adam's first and second
 * moments (HOST float[n_params] each; any may be NULL to skip it), the number of Adam steps
 * taken (NULL to skip) and the normalisation (HOST float[8] or NULL).  Synchronous. */
int tr_mlp_get_state(tr_ctx *ctx, const tr_mlp *mlp, float *params_host, float *adam_m_host,
                     float *adam_v_host, int64_t *steps, float *norm_host);
/* Restores a state read by tr_mlp_get_state into a network (NULL moments restart them at
 * zero); the next tr_mlp_train_step is Adam step steps + 1, with that step's bias
 * correction.  TR_EINVAL for NULL params or negative steps.  Synchronous. */
int tr_mlp_set_state(tr_ctx *ctx, tr_mlp *mlp, const float *params_host, const float *adam_m_host,
                     const float *adam_v_host, int64_t steps);
/* Forward only: x device float[n][3] (already normalised) -> y device float[n]; n = 0 does
 * nothing (x and y may then be NULL). */
int tr_mlp_forward(tr_ctx *ctx, const tr_mlp *mlp, int64_t n, const float *x, float *y);
/* Loss and gradients of the mean squared error for one batch: grad device
 * float[n_params] (overwritten), loss device float[1]. */
int tr_mlp_grad(tr_ctx *ctx, const tr_mlp *mlp, int64_t n, const float *x, const float *y,
                float *grad, float *loss);
/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on the batch; loss device
 * float[1] or NULL. */
int tr_mlp_train_step(tr_ctx *ctx, tr_mlp *mlp, int64_t n, const float *x, const float *y,
                      float lr, float *loss);

/* Ionising side of the stellar sources (Sec. 7.2).  Per star: T_int = (L_int / (4 pi
 * sigma r^2))^(1/4), T_acc = (L_acc / (f_fill 4 pi sigma r^2))^(1/4), gamma(T) = fraction of a
 * black body's power above the Lyman limit (t_lyc = h nu_LyC / k, 157 821 K for 13.6 eV),
 * L_uv = gamma(T_int) L_int + gamma(T_acc) L_acc, L_ir = L_int + L_acc - L_uv (the L_IR
 * that tr_build_tree takes).  All arrays device double[n]; FP64. */
int tr_star_luminosity_split(tr_ctx *ctx, int n, const double *L_int, const double *L_acc,
                             const double *r_star, double f_fill, double sigma, double t_lyc,
                             double *L_uv, double *L_ir);

/* UV radiation pressure (App. C) for an ionising photon number flux n_ph (photons per unit
 * area and time, from the ionising-radiation solver) of mean energy e_ph along the unit
 * vector u_ph: momentum rates per volume on dust sigma_d n (e_ph/c) n_ph, on neutral
 * hydrogen sigma_h (1 - x) n (e_ph/c) n_ph and on ionised hydrogen alpha_b (x n)^2 (e_ph/c)
 * (recombinations balanced by absorptions), n = rho / mu_mh, x = ionised fraction.
 * a_uv = (their sum) u_ph / rho.  rho, x_ion, n_ph: device float[n]; u_ph, a_uv: device
 * float[3][n]; parts: device float[3][n] (dust, H, H+) or NULL. */
typedef struct tr_uv_params {
    double e_ph;    /* mean ionising photon energy */
    double sigma_d; /* dust cross section per hydrogen nucleus (1.5e-21 cm^2 in the paper) */
    double sigma_h; /* hydrogen photoionisation cross section */
    double alpha_b; /* case-B recombination coefficient */
    double mu_mh;   /* mass per hydrogen nucleus (1.4 m_H) */
    double c;
} tr_uv_params;
int tr_uv_rad_pressure(tr_ctx *ctx, int64_t n, const float *rho, const float *x_ion, const float *n_ph,
                       const float *u_ph, const tr_uv_params *p, float *a_uv, float *parts);

/* Context: one HIP device and stream (hipStream_t passed as void*, NULL = null stream). */
int tr_ctx_create(tr_ctx **out, int device, void *stream);
void tr_ctx_destroy(tr_ctx *ctx);
int tr_ctx_set_stream(tr_ctx *ctx, void *stream);
/* Input validation (off by default): when on, tr_build_tree checks every cell's rho, kappa (if
 * given) and t_dust and fails with TR_EINVAL, building nothing, if any is negative, infinite or
 * NaN (the paper's densities, opacities and temperatures are finite and non-negative, Sec. 2,
 * 4.1).  The check is one extra kernel before the build's single synchronisation. */
int tr_ctx_set_validation(tr_ctx *ctx, int on);
const char *tr_last_error(const tr_ctx *ctx);
/* Wait for the stream and report latched device-side failures (TR_EOVERFLOW). */
int tr_sync(tr_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
