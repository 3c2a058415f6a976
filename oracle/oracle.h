/*
 * TreeRay/RadPressure FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow reference of the hot path (tree build, ray mapping and integration,
 * ray finalisation, radiation-pressure force, dust equilibrium, MLP) written from
 * Klepitko et al. (MNRAS 2023, arXiv 2204.09072).  Only the tests, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code, header, table or constant generator with the HIP library.
 */
#ifndef TREERAY_ORACLE_H
#define TREERAY_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_tree or_tree;

/* Tree build (Sec. 4.1 and App. A).  blocks: [n_blk][4] = (level, bi, bj, bk) of leaf
 * blocks of 8^3 cells; cell arrays block-major, local cell index ci + 8cj + 64ck.
 * kappa may be NULL (Planck-mean opacity from t_dust, Sec. 2).  stars: [n_star][4]
 * = (x, y, z, L_IR).  Returns NULL on invalid input. */
or_tree *or_build_tree(int nb, int max_level, int n_blk, const int32_t *blocks,
                       const double *x0, double box_len, const float *rho,
                       const float *kappa, const float *t_dust, int n_star,
                       const double *stars, double sigma);
void or_tree_free(or_tree *t);

/* what: 0 n_node, 1 n_leaf, 2 depth of finest cells, 3 root edge (lattice units),
 *       4 number of ray bins for isolated boundaries, 5 n_cells */
int64_t or_tree_count(const or_tree *t, int what);
double or_tree_u_len(const or_tree *t);

/* Node export in the library's documented layout (depth-major, Morton inside a depth).
 * geo [n][4] = (gx, gy, gz, first_child or -1); meta[n] = depth | mask<<4 | leaf<<12 |
 * (thick content)<<13;
 * q [n][4]: leaf (L signed, A, S, 0), h-node (L_thin, LV_thick, A_thin, A_thick);
 * vthick[n]; pcol [n][3] (2^-8 lattice units); leaf_cell[n] (-1 for h-nodes). */
void or_tree_export(const or_tree *t, int32_t *geo, uint32_t *meta, float *q,
                    float *vthick, int32_t *pcol, int64_t *leaf_cell);
/* FP64 sums per node [n][6] = (L_thin, LV_thick, A_thin, A_thick, V_thick, xi). */
void or_tree_export_f64(const or_tree *t, double *out);

/* HEALPix NESTED (Gorski et al. 2005) */
void or_pix2vec(int n_side, int pix, double *v);
int or_vec2pix(int n_side, double x, double y, double z);
/* direction-cell table for the angular kernel: [6][M][M] pixel ids */
void or_cube_table(int n_side, int M, int32_t *out);
/* tabulated angular kernel: [6][M][M][15 distance classes][9] = pixels 0..3, counts 0..3
 * (out of 64), flag of keys reaching more than 4 pixels */
void or_alpha_table(int M, const int32_t *pixtab, int32_t *out);

typedef struct {
    int n_side;
    int theta_num, theta_den;   /* accept a node when edge/distance < num/den */
    int cube_m;                 /* direction cells per cube-face edge */
    int merge;                  /* merge segments spanned by thick material */
    double j_bg;                /* background intensity at the ray ends */
    int orient;                 /* ray-set orientation: 0..47 (signed axis permutation
                                   applied to node offsets), -1 = drawn per target cell */
    unsigned int orient_seed;   /* seed of the per-target draw */
    int alpha_table;            /* 1: tabulated angular kernel for nodes >= 8 edges away */
} or_params;

/* Trace every target in `cells` (cell indices; NULL = all n cells, in cell order).
 * J[n], F[n][3] (FP64), counters[n][3] = (leaves accepted, h-nodes accepted, opened)
 * may be NULL.  n_threads <= 0 uses OpenMP's default. */
int or_trace(const or_tree *t, const or_params *p, int64_t n, const int64_t *cells,
             double *J, double *F, int64_t *counters, int n_threads);

/* One target, with its ray bins [N_pix][N_b+1][6] (L_thin, A_thin, L_thick, A_thick,
 * V_thick, Q), merge flags [N_pix][N_b+1], per-ray flux F^h and total thin depth.
 * brute != 0 maps every leaf directly (no tree walk, no opening test). */
int or_trace_one(const or_tree *t, const or_params *p, int64_t cell, int brute,
                 double *bins, uint8_t *flags, double *Fh, double *tau_thin_tot,
                 double *J, double *F);

/* Integrate one ray from given bins (same layout, one ray): returns F^h. */
double or_integrate_ray(int n_side, int n_bins, const double *bins, const uint8_t *flags,
                        double j_bg);

/* Direct ray marching through a uniform n^3 grid over [0, box)^3 without the tree (the
 * brute-force reference of the method's end-to-end error).  kr = rho kappa per length and
 * B = source function, dense [(i n + j) n + k]; returns the intensity along unit vector u
 * from point p, *tau_out the optical depth to the grid's edge.  skip_own: the start cell
 * neither absorbs nor emits. */
double or_march(int n, double box, const double *kr, const double *B, const double *p,
                const double *u, int skip_own, double *tau_out);
/* Mean over the 4^sub NESTED sub-pixels of every pixel of the N_side = ns set: J[n_pt]
 * (mean intensity) and absorbed[n_pt] (mean of 1 - e^-tau); either may be NULL. */
void or_march_mean(int n, double box, const double *kr, const double *B, int64_t n_pt,
                   const double *pts, int ns, int sub, int skip_own, double *J, double *absorbed);
/* pixel ids of n directions [n][3] */
void or_vec2pix_many(int n_side, int64_t n, const double *v, int32_t *out);

/* Radiation-pressure acceleration a[n][3] and trapped pressure p_src[n] (Sec. 4.5). */
void or_rad_force(const or_tree *t, const float *rho, const float *kappa,
                  const float *t_dust, const double *F, double c, double *a, double *p_src);

/* Dust equilibrium temperature (Sec. 4.6, App. E), bracketed bisection in FP64. */
void or_dust_eq(int64_t n, const double *rho, const double *u_rad, const double *t_gas,
                double sigma, double c, double c_gd, double xi, double *t_dust, int *iters);
double or_dust_residual(double T, double rho, double u_rad, double t_gas, double sigma,
                        double c, double c_gd, double xi);

/* Lyman-continuum fraction of a black body (Sec. 7.2), t_lyc = h nu_LyC / k. */
double or_lyman_fraction(double T, double t_lyc);
/* Split of internal and accretion luminosities into ionising L_uv and non-ionising L_ir
 * (Sec. 7.2; hot-spot filling factor f_fill). */
void or_luminosity_split(int n, const double *L_int, const double *L_acc, const double *r_star,
                         double f_fill, double sigma, double t_lyc, double *L_uv, double *L_ir);
/* UV radiation pressure (App. C): acceleration a[n][3] and, if parts != NULL, the momentum
 * rates per volume on dust, H and H+ [n][3]. */
void or_uv_rad_pressure(int64_t n, const double *rho, const double *x_ion, const double *nph,
                        const double *uph, double e_ph, double sigma_d, double sigma_h, double alpha_b,
                        double mu_mh, double c, double *a, double *parts);

/* MLP 3 -> H -> H -> 1 (ReLU hidden layers), FP64 forward and backward for a batch; parameter
 * layout W1[H][3] b1[H] W2[H][H] b2[H] W3[H] b3.  round_bf16 != 0 rounds each layer's
 * input activations to bfloat16 (as the GPU's MFMA operands).  Returns the mean
 * squared error; grad (same layout) may be NULL; out[n] may be NULL. */
double or_mlp(int H, const double *params, int64_t n, const double *x, const double *y,
              int round_bf16, double *out, double *grad);

#ifdef __cplusplus
}
#endif
#endif
