/*
 * gap.h -- C ABI of the MI355X (gfx950) GAP regression hot path.
 *
 * Sparse Gaussian-process regression for Gaussian Approximation Potentials
 * with the polynomial dot-product kernel k(x, x') = delta^2 (x . x')^zeta
 * (Klawohn et al., arXiv:2310.03921, Sec. "Theory" and Sec. "Regression").
 *
 * Conventions shared by every call
 * --------------------------------
 * - All array arguments are DEVICE pointers on the handle's device, owned by
 *   the caller, unless a comment says "host".  The library owns only the
 *   workspace attached to the handle (grown on demand, freed by gap_destroy).
 * - Work is enqueued on the handle's HIP stream.  Every call is asynchronous
 *   except gap_fit, gap_lstsq and gap_sync, which wait for the stream because
 *   they report conditions found on the device (NOT_PD, RANK, bad indices).
 * - Argument errors are returned before anything is enqueued; the message is
 *   kept in the handle (gap_last_error).  Device-side index errors (a pair
 *   target outside [0, n_atoms)) drop the offending pair and are reported as
 *   GAP_E_INVALID by the next synchronising call.
 * - Row-major arrays have a leading dimension ld >= the row length; every
 *   leading dimension of a floating-point row-major array must be a multiple
 *   of 4 elements and the base pointer 32-byte aligned (vector loads).
 *   Elements between the row length and ld are never read.
 * - Column-major matrices (K_MM, K_NM, the least-squares matrix) have ld >=
 *   the number of rows.
 * - Observation rows of K_NM: row c < n_cfg is the total energy of
 *   configuration c; row n_cfg + 3 j + alpha is force component alpha on atom
 *   j.  Force rows carry the minus sign of F = -dE/dr.
 * - Only integer zeta >= 1 is supported (descriptor dot products can be
 *   negative); anything else returns GAP_E_UNSUPPORTED.
 */
#ifndef GAP_H
#define GAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GAP_OK = 0,
  GAP_E_INVALID = -1,     /* bad argument or bad index data                 */
  GAP_E_NOT_PD = -2,      /* K_MM + jitter I is not positive definite        */
  GAP_E_RANK = -3,        /* R of the least-squares QR has a zero pivot      */
  GAP_E_NOMEM = -4,       /* workspace allocation failed                     */
  GAP_E_HIP = -5,         /* HIP runtime error                               */
  GAP_E_UNSUPPORTED = -6  /* valid request this build does not implement     */
} gap_status;

/* Arithmetic of the descriptor / Jacobian contractions.
 * GAP_FP64:   FP64 MFMA throughout.
 * GAP_BF16X3: each FP32 operand x is split into hi = bf16(x), lo = bf16(x - hi);
 *             products hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32
 *             accumulation (lo*lo dropped).  Scales, reductions and outputs
 *             stay FP64. */
typedef enum { GAP_FP64 = 0, GAP_BF16X3 = 1 } gap_precision;

typedef enum { GAP_DT_F32 = 0, GAP_DT_F64 = 1 } gap_dtype;

typedef struct gap_handle gap_handle;

/* A batch of atomic configurations: the descriptors x_i of every atom and the
 * descriptor derivatives with "pointers" to the atoms they belong to
 * (Sec. "Regression", last paragraph; Sec. "Program structure").
 *   cfg_ptr  [n_cfg+1]   int64  atoms of configuration c: cfg_ptr[c] .. cfg_ptr[c+1]-1
 *                               (cfg_ptr[0] = 0, cfg_ptr[n_cfg] = n_atoms, non-decreasing)
 *   desc     [n_atoms][ld_desc]  descriptor rows, f32 or f64
 *   pair_ptr [n_atoms+1] int64  source-major CSR of neighbour pairs (i, k):
 *                               pairs of atom i are pair_ptr[i] .. pair_ptr[i+1]-1,
 *                               pair_ptr[n_atoms] = n_pairs
 *   pair_j   [n_pairs]   int32  global atom index j(i, k) the pair points at
 *   jac      [n_pairs][3][ld_jac]  d desc_i / d r_{j(i,k), alpha}, f32 or f64
 *                               (may be NULL when no force rows / forces are asked) */
typedef struct {
  int64_t n_cfg, n_atoms, n_pairs, D;
  const int64_t *cfg_ptr;
  const void *desc;
  gap_dtype desc_dt;
  int64_t ld_desc;
  const int64_t *pair_ptr;
  const int32_t *pair_j;
  const void *jac;
  gap_dtype jac_dt;
  int64_t ld_jac;
} gap_atoms;

/* Sparse (representative) points x_m, m < M, row-major FP64 [M][ld_x],
 * and the kernel hyperparameters: zeta (soap_exponent) and delta
 * (energy_scale, the GP standard deviation). */
typedef struct {
  int64_t M, D, ld_x;
  const double *X;
  int zeta;
  double delta;
} gap_sparse;

/* Host-side report of gap_fit. */
typedef struct {
  double resid_norm[8];  /* ||A^T (b - A c)|| after the solve and after each refinement step */
  double min_abs_rdiag;  /* min_k |R_kk| of the QR factor */
  double max_abs_rdiag;  /* max_k |R_kk| */
  int refine_done;       /* refinement steps carried out */
} gap_fit_info;

/* Create a handle bound to HIP device `device` and HIP stream `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream).  Every call is ordered on
 * that stream; a call may also run part of its work on a side stream of the
 * handle (default priority), forked from and joined back to the caller's
 * stream with events inside the call.  Fails with GAP_E_HIP if the device is
 * missing or is not gfx950, or if the side stream cannot be created. */
gap_status gap_create(gap_handle **h, int device, void *hip_stream);
gap_status gap_destroy(gap_handle *h);
/* Message of the last error on this handle ("" if none).  Valid until the
 * next call on the handle. */
const char *gap_last_error(const gap_handle *h);
/* Wait for the handle's stream and report deferred device-side errors. */
gap_status gap_sync(gap_handle *h);

/* Cap, in bytes, on the optional workspace the handle may take for speed
 * (0, the default: no cap).  Today that is the Jacobians of a BF16X3
 * gap_build_knm with D <= 256 split once into hi / lo halves (4 bytes per
 * entry, at most 16 GB), which the call otherwise takes whenever they fit in
 * 85% of the free device memory; under the cap the rows are split in registers
 * instead (same results, more time).  Required workspace is not capped. */
gap_status gap_set_workspace_limit(gap_handle *h, size_t bytes);

/* Workspace bytes the handle will hold for a fit of `atoms` with `sp`
 * (K_NM and the least-squares matrix excluded: those are caller buffers);
 * the equivalent of a dry run (cf. the gap_fit `dryrun` argument). */
gap_status gap_workspace_query(gap_handle *h, const gap_atoms *atoms, const gap_sparse *sp,
                               size_t *bytes);

/* Target-major view of the pair list that the operator L-hat needs to
 * accumulate force observations (Sec. "Theory", definition of L-hat):
 *   tgt_ptr  [n_atoms+1] int64, tgt_pair [n_pairs] int32 -- the pairs pointing
 *   at atom j are tgt_pair[tgt_ptr[j] .. tgt_ptr[j+1]-1] in increasing pair order.
 * Pairs whose target is out of range are left out (and reported). */
gap_status gap_pair_transpose(gap_handle *h, const gap_atoms *atoms, int64_t *tgt_ptr,
                              int32_t *tgt_pair);

/* K_MM[m][m'] = delta^2 (x_m . x_m')^zeta, column-major M x M with leading
 * dimension ld >= M (no jitter).  Exactly symmetric: each off-diagonal value
 * is computed once and stored at both positions.
 * (Sec. "Theory", definition of K_MM after eq. GP_L.) */
gap_status gap_build_kmm(gap_handle *h, const gap_sparse *sp, double *Kmm, int64_t ld);

/* L-hat K_NM, column-major, (n_cfg + 3 n_atoms) rows x M columns, ld >= rows:
 *   energy row c:        sum_{i in c} delta^2 (d_i . x_m)^zeta
 *   force row (j,alpha): - sum_{(i,k): j(i,k)=j} delta^2 zeta (d_i . x_m)^(zeta-1) J[(i,k),alpha] . x_m
 * (Sec. "Theory": eq. 1, eq. epsilon, the derivative rows of K_NM.)
 * Pairs may point at any atom of the batch.  `prec` selects the contraction
 * arithmetic (GAP_BF16X3 requires jac_dt / desc_dt in {F32, F64}; values are
 * rounded to FP32 before the split). */
gap_status gap_build_knm(gap_handle *h, const gap_atoms *atoms, const gap_sparse *sp,
                         gap_precision prec, double *Knm, int64_t ld);

/* Per-species GP block (Sec. "Theory", eq. 1: the total energy is a sum over
 * descriptor types of local energies, each type a GP of its own; a descriptor
 * defined for one central species, as in the multi-species models of the
 * "Practical examples", gives one such GP per species).  The rows of
 * gap_build_knm with only the atoms of species z as centres:
 *   energy row c:        sum_{i in c, species[i] = z} delta^2 (d_i . x_m)^zeta
 *   force row (j,alpha): - sum_{(i,k): j(i,k)=j, species[i] = z} delta^2 zeta (d_i . x_m)^(zeta-1)
 *                          J[(i,k),alpha] . x_m
 * Targets j of any species receive forces.  species [n_atoms] int32 device.
 * A model of several species puts the blocks side by side (columns of each
 * block's sparse points, K = Knm + M_prev * ld) in one design buffer or fold
 * block, with K_MM block-diagonal, and fits them together (gap_fit without
 * refinement, or the gap_fold_* calls).  Same layout, precision and errors as
 * gap_build_knm.  Asynchronous. */
gap_status gap_build_knm_species(gap_handle *h, const gap_atoms *atoms, const gap_sparse *sp,
                                 gap_precision prec, const int32_t *species, int32_t z,
                                 double *Knm, int64_t ld);

/* Two-body descriptor with the squared-exponential kernel, for models of
 * several descriptors (Sec. "Descriptors based on interatomic distances":
 * distance_2b, the pair distance as descriptor, the kernel multiplied by the
 * cosine cutoff f_cut(r) of width d below r_cut; Sec. "Regression": k_SE).
 * Each directed pair p = (i, k) of `atoms` (pair_ptr / pair_j) is an instance
 * with r = |pair_r[p]| (pair_r: displacement r_j - r_i, [n_pairs][3] FP64
 * device) that carries half of its bond's energy (a full neighbour list holds
 * each bond twice):
 *   k(r, x) = delta^2 f_cut(r) f_cut(x) exp(-(r - x)^2 / (2 theta^2)),
 *   energy row c:         sum_{p in c} k(r_p, x_m) / 2,
 *   force row (a, alpha): -d/dr_a,alpha of that sum.
 * The rows have gap_build_knm's layout (n_cfg energies, then 3 per atom), so
 * a two-body block of columns sits beside a dot-product block in one design
 * buffer or fold block (K = Knm + M1 * ld), with K_MM block-diagonal.  Only
 * cfg_ptr, pair_ptr and pair_j of `atoms` are read. */
typedef struct {
  int64_t M;         /* sparse distances */
  const double *x;   /* [M] device */
  double delta;      /* energy scale */
  double theta;      /* length scale > 0 */
  double r_cut;      /* cutoff > 0 */
  double cut_width;  /* transition width, 0 < cut_width <= r_cut */
} gap_se2b;
/* L-hat K_NM block of the two-body descriptor: column-major (n_cfg + 3 n_atoms)
 * x M, ld >= rows.  Asynchronous. */
gap_status gap_build_2b_rows(gap_handle *h, const gap_atoms *atoms, const double *pair_r,
                             const gap_se2b *k2, double *K, int64_t ld);
/* K_MM[m][m'] = k(x_m, x_m'), column-major M x M, ld >= M, exactly symmetric. */
gap_status gap_build_kmm_2b(gap_handle *h, const gap_se2b *k2, double *Kmm, int64_t ld);
/* The two-body part of a prediction with coefficients c [M]: configuration
 * energies e_cfg [n_cfg] and forces [n_atoms][3] (FP64 device, either may be
 * NULL), written (add the dot-product part of gap_predict for the model's
 * total).  Asynchronous. */
gap_status gap_predict_2b(gap_handle *h, const gap_atoms *atoms, const double *pair_r,
                          const gap_se2b *k2, const double *c, double *e_cfg, double *forces);

/* Virial rows: the nine components of a configuration's virial stress as
 * observations (Sec. "Theory": targets are totals of local energies or of
 * their partial derivatives, virial stresses among them; sigma_virial
 * regularises them).  The paper gives no formula; the library takes the
 * strain derivative.  With r_p the displacement r_j(p) - r_i of pair p = (i, k)
 * (periodic image included) and a homogeneous strain eps acting as
 * r_p -> (I + eps) r_p,
 *   W_alpha,beta(c) = - sum_{p in c} r_p,alpha dE/dr_j(p),beta   (= - dE/d eps_beta,alpha)
 * so row 9 c + 3 alpha + beta, column m of Kv is
 *   - sum_{p in c} r[p][alpha] delta^2 zeta (d_i . x_m)^(zeta-1) J[p][beta] . x_m.
 * pair_r [n_pairs][3] FP64 device.  Kv column-major 9 n_cfg x M, ld >= 9 n_cfg
 * (it may point into a design buffer below other rows, or into a fold
 * state's block area).  Asynchronous.  FP64 contraction. */
gap_status gap_build_virial_rows(gap_handle *h, const gap_atoms *atoms, const gap_sparse *sp,
                                 const double *pair_r, double *Kv, int64_t ld);

/* Local-property rows (Sec. "Local Property": a per-atom property such as a
 * core-electron binding energy learned directly; a mask marks the atoms that
 * carry one, so L-hat for such an observation selects a single atom):
 *   K[r][m] = delta^2 (d_i . x_m)^zeta,  i = atom_idx[r],
 * column-major n_local x M with ld >= n_local (K may point into a design
 * buffer below other rows, or into a fold state's block area).  atom_idx
 * [n_local] int32 device: the compacted mask, 0 <= atom_idx[r] < n_atoms.
 * Only the descriptors of `atoms` are read (jac may be NULL).  The predicted
 * property is gap_predict's e_atom; per-species offsets are the caller's
 * (subtract them from the targets).  Asynchronous; an index out of range gives
 * a zero row and GAP_E_INVALID at the next synchronising call. */
gap_status gap_build_local_rows(gap_handle *h, const gap_atoms *atoms, const gap_sparse *sp,
                                const int32_t *atom_idx, int64_t n_local, double *K, int64_t ld);

/* Least-squares solve of min ||A x - b|| by blocked Householder QR and back
 * substitution, x = R^-1 (Q^T b)[0:n] (Sec. "Theory", QR route).
 * A is column-major m x (n+1) with ld >= m, m >= n; column n holds b.
 * A is overwritten by the Householder vectors, R and Q^T b.  x: [n].
 * Returns GAP_E_RANK if some R_kk is zero or not finite.
 * `rdiag_minmax` (host, may be NULL) receives min and max |R_kk|.  Synchronous. */
gap_status gap_lstsq(gap_handle *h, double *A, int64_t ld, int64_t m, int64_t n, double *x,
                     double *rdiag_minmax);

/* Fit the sparse-GPR coefficients c (Sec. "Theory"):
 *   A = [Sigma^-1/2 L-hat K_NM ; U_MM],  b = [Sigma^-1/2 y ; 0],
 *   K_MM + jitter I = U^T U (upper Cholesky),  c = R^-1 Q^T b.
 * A: column-major buffer with ld >= n_rows + M and M + 1 columns; on entry
 *    rows [0, n_rows) of columns [0, M) hold L-hat K_NM (as written by
 *    gap_build_knm with the same ld); the whole buffer is overwritten.
 * Kmm [M x M] col-major (ld = M), y [n_rows], sigma [n_rows] > 0, jitter >= 0.
 * refine_steps > 0 (requires `train`): after the solve, up to that many steps of
 *    r = b - A_exact c,  R^T R dc = A_exact^T r,  c += dc
 *    with A_exact applied matrix-free in FP64 from `train` and `sp`
 *    (iterative refinement of the mixed-precision form; the residual is exact
 *    FP64 so it removes the assembly error of a BF16X3 K_NM).  Each step
 *    contracts the error of c by about the same factor, so after step k >= 2
 *    the error left is about |dc_k|^2 / |dc_k-1| (relative to |c|); the steps
 *    stop once that is below 1e-14.  info->refine_done counts the steps taken,
 *    info->resid_norm[0 .. refine_done] the |A_exact^T r| before each and after
 *    the last (that last one costs a whole residual pass and only reports;
 *    gap_set_fit_report(h, 0) skips it, leaving resid_norm[refine_done] NaN).
 * c: [M] output.  info: host, may be NULL.  Synchronous.
 * Returns GAP_E_NOT_PD if the Cholesky of K_MM + jitter I fails. */
gap_status gap_fit(gap_handle *h, double *A, int64_t ld, int64_t n_rows, const double *Kmm,
                   const double *y, const double *sigma, double jitter, const gap_atoms *train,
                   const gap_sparse *sp, int refine_steps, double *c, gap_fit_info *info);

/* Whether gap_fit computes the residual after its last refinement step
 * (default 1).  That residual only fills info->resid_norm[refine_done]; it
 * changes neither c nor the number of steps, so a caller that does not read
 * it can skip one FP64 residual pass per fit with 0. */
gap_status gap_set_fit_report(gap_handle *h, int final_residual);

/* Predictive variance of the local energies (Sec. "Regression": gp_predict
 * also returns the variances the GPR predicts).  The paper gives no formula;
 * the library takes the sparse (projected-process) GP form that goes with the
 * coefficients of eq. GP_L:
 *   var_i = k(d_i, d_i) - k_i^T (K_MM + jitter I)^-1 k_i
 *           + k_i^T (K_MM + jitter I + K_MN Sigma^-1 K_NM)^-1 k_i,
 *   k_i[m] = delta^2 (d_i . x_m)^zeta,
 * evaluated as ||U^-T k_i||^2 and ||R^-T k_i||^2 with U the upper Cholesky factor
 * of K_MM + jitter I and R the fit's triangular factor (R^T R = A^T A): the
 * upper triangle of the leading M x M block of A after gap_fit, or of a fold
 * state T (col-major, ld ldr >= M; entries below the diagonal are not read).
 * Kmm [M x M] col-major (ld = M), the same jitter as the fit.  var [n_atoms]
 * device FP64.  Only the descriptors of `atoms` are read.  Synchronous;
 * GAP_E_NOT_PD if the Cholesky fails, GAP_E_RANK if R has a zero pivot. */
gap_status gap_predict_variance(gap_handle *h, const gap_atoms *atoms, const gap_sparse *sp,
                                const double *Kmm, double jitter, const double *R, int64_t ldr,
                                double *var);

/* CUR selection of sparse points among the atoms' descriptors (Sec. "Sparse
 * point selection": cur_points, a CUR decomposition of the data points after
 * Mahoney & Drineas, whose column choice rests on leverage scores).  With the
 * rank parameter taken as the full rank of the descriptor matrix D (n_atoms x
 * D), regularised by jitter, the leverage of atom i is
 *   l_i = d_i^T (D^T D + jitter I)^-1 d_i.
 * u == NULL: the n_sparse atoms of largest leverage.  u [n_atoms] device,
 * uniform in (0, 1]: exact-size weighted sampling without replacement with
 * weights l_i (keys log(u_i) / l_i, largest first; Efraimidis & Spirakis).
 * Ties go to the smaller atom index.  out_idx [n_sparse] int32 device, in
 * decreasing key order; leverage [n_atoms] device FP64 (may be NULL).  Only
 * the descriptors of `atoms` are read.  Synchronous; GAP_E_NOT_PD if
 * D^T D + jitter I is not positive definite (use jitter > 0 for descriptor
 * sets of lower rank). */
gap_status gap_select_cur(gap_handle *h, const gap_atoms *atoms, int64_t n_sparse, double jitter,
                          const double *u, int32_t *out_idx, double *leverage);

/* Streamed fit: the least-squares problem of gap_fit folded one block of
 * observation rows at a time, so that A is never held whole.  Sec. "Theory"
 * gives the QR route; Sec. "Program structure" splits the configurations, and
 * so the rows of L-hat K_NM (its main memory cost), into groups built apart.
 * Row order does not change a least-squares problem, and the triangular
 * factor of [T_prev ; block] is that of all rows seen (T^T T = [A | b]^T [A | b]).
 * State T: column-major buffer of M + 1 columns with ld >= M + 1 + n_rows of
 * every fold, ld % 4 == 0, 32-byte aligned.  Rows [0, M + 1) hold the upper
 * triangular factor of the augmented matrix [A_seen | b_seen] of the rows
 * folded so far (R of A_seen, then (Q^T b)[0:M] in column M and, in the
 * corner T[M][M], the norm of the least-squares residual).  Rows
 * [M + 1, M + 1 + n_rows) are the block area: before gap_fold_rows the caller
 * writes the block's L-hat K_NM rows there, columns [0, M) (gap_build_knm with
 * Knm = T + M + 1 and the same ld).  Every call is ordered on the handle's
 * stream; gap_fold_init and gap_fold_solve wait for it, gap_fold_rows does not
 * (device-side errors of a fold surface at the next synchronising call).
 *
 * gap_fold_init: T = [U 0; 0 0], U the upper Cholesky factor of K_MM + jitter I
 *   (the rows U_MM of A).  Kmm [M x M] col-major (ld = M).  Rows >= M + 1
 *   are not touched.  Returns GAP_E_NOT_PD if the Cholesky fails. */
gap_status gap_fold_init(gap_handle *h, double *T, int64_t ld, int64_t M, const double *Kmm,
                         double jitter);
/* gap_fold_rows: fold the n_rows block rows (n_rows >= 0; 0 is a no-op):
 *   scale row r by 1 / sigma[r], put y[r] / sigma[r] in column M, and replace
 *   T by the triangular factor of [T ; block] (Householder QR of the stacked
 *   M + 1 + n_rows rows, then the corner norm).  y, sigma [n_rows] device,
 *   sigma > 0.  The block area is overwritten (Householder vectors). */
gap_status gap_fold_rows(gap_handle *h, double *T, int64_t ld, int64_t M, int64_t n_rows,
                         const double *y, const double *sigma);
/* gap_fold_solve: c = R^-1 (Q^T b)[0:M] from the state (device c [M]).
 *   lsq_resid (host, may be NULL) = |T[M][M]| = ||b - A c|| over all rows folded.
 *   rdiag_minmax (host, may be NULL) = min and max |R_kk|.
 *   Returns GAP_E_RANK if some R_kk is zero or not finite. */
gap_status gap_fold_solve(gap_handle *h, const double *T, int64_t ld, int64_t M, double *c,
                          double *lsq_resid, double *rdiag_minmax);

/* Refinement by batches of observation rows (Sec. "Theory", least-squares
 * form; the residual is taken in FP64 from the exact rows while R may come from
 * approximate ones, e.g. BF16X3 rows folded by gap_fold_rows).  One step over
 * the whole training set, with r = b - A c the residual of the stacked system
 * [Sigma^-1/2 L-hat K_NM ; U] c = [Sigma^-1/2 y ; 0]:
 *   g = 0 (device, M doubles); gap_refine_rows for every batch;
 *   gap_refine_solve, which adds the rows U and computes c += (R^T R)^-1 g.
 *
 * gap_refine_rows: for the batch a's rows (its energy rows, then three force
 *   rows per atom: the row order of gap_build_knm), with K the exact FP64 rows
 *   computed matrix-free from a's descriptors and Jacobians (needs jac) and
 *   r = Sigma^-1/2 (y - K c):
 *     g[0:M] += K^T Sigma^-1/2 r,   rr[0] += r . r   (rr may be NULL).
 *   c [M], y and sigma [n_cfg + 3 n_atoms], g, rr: device FP64.  D <= 2048.
 *   Asynchronous on the handle's stream; a batch without rows is a no-op. */
gap_status gap_refine_rows(gap_handle *h, const gap_atoms *a, const gap_sparse *sp,
                           const double *c, const double *y, const double *sigma, double *g,
                           double *rr);
/* gap_refine_weights / gap_refine_rows_s: the same step with the batch's
 *   exact FP64 kernel-gradient scale kept by the caller between passes,
 *     S[i][m] = delta^2 zeta (d_i . x_m)^(zeta-1),
 *   row-major [n_atoms][ldS] FP64 device (ldS >= M, ldS % 4 == 0, 32-byte
 *   aligned; 8 n_atoms ldS bytes), so that a pass over a batch needs no
 *   descriptor product of its own.  gap_refine_weights writes S of batch a
 *   (columns M .. ldS - 1 zero); gap_refine_rows_s is gap_refine_rows with that
 *   S (the same batch and sparse points).  Both asynchronous. */
gap_status gap_refine_weights(gap_handle *h, const gap_atoms *a, const gap_sparse *sp, double *S,
                              int64_t ldS);
gap_status gap_refine_rows_s(gap_handle *h, const gap_atoms *a, const gap_sparse *sp,
                             const double *S, int64_t ldS, const double *c, const double *y,
                             const double *sigma, double *g, double *rr);
/* gap_refine_solve: adds the regulariser rows' share U^T (0 - U c) =
 *   -(K_MM + jitter I) c to g, then solves R^T R dc = g and sets c += dc; g is
 *   overwritten by dc.  R: the upper triangle of the first M columns of a
 *   factor with leading dimension ldr >= M (A after gap_fit, or a fold state
 *   T).  Kmm [M x M] col-major (ld = M), c and g [M]: device.  Synchronous.
 *   Returns GAP_E_RANK if some R_kk is zero or not finite. */
gap_status gap_refine_solve(gap_handle *h, const double *R, int64_t ldr, int64_t M,
                            const double *Kmm, double jitter, double *g, double *c);

/* Predict with coefficients c [M] (eq. epsilon and the chain rule for forces):
 *   e_atom [n_atoms]      eps_i = sum_m c_m delta^2 (d_i . x_m)^zeta
 *   e_cfg  [n_cfg]        sum of eps_i over the configuration
 *   dEdd   [n_atoms][D]   g_i = d eps_i / d d_i (row-major, ld = D)
 *   forces [n_atoms][3]   F_j = - sum_{(i,k): j(i,k)=j} J[(i,k)]^T g_i   (needs jac)
 * All outputs FP64; any may be NULL. */
gap_status gap_predict(gap_handle *h, const gap_atoms *atoms, const gap_sparse *sp,
                       const double *c, gap_precision prec, double *e_atom, double *e_cfg,
                       double *dEdd, double *forces);

/* gap_predict of the per-species GP block of species z (see
 * gap_build_knm_species): eps_i as gap_predict for atoms with species[i] = z,
 * 0 for the others; e_cfg, dEdd and forces follow from those eps_i.  The
 * model's prediction is the sum of its species blocks' outputs.
 * species [n_atoms] int32 device.  Asynchronous. */
gap_status gap_predict_species(gap_handle *h, const gap_atoms *atoms, const gap_sparse *sp,
                               const double *c, gap_precision prec, const int32_t *species,
                               int32_t z, double *e_atom, double *e_cfg, double *dEdd,
                               double *forces);

/* Backward of e_atom = predict(desc, X, c) for an upstream gradient g_e [n_atoms]
 * (differentiation of eq. epsilon; (d_i . x_m)^(zeta-1) is recomputed):
 *   d_desc [n_atoms][D] = g_e[i] g_i
 *   d_c    [M]          = sum_i g_e[i] delta^2 (d_i . x_m)^zeta
 *   d_X    [M][D]       = c_m sum_i g_e[i] delta^2 zeta (d_i . x_m)^(zeta-1) d_i
 * All FP64 row-major (ld = D); any may be NULL. */
gap_status gap_predict_backward(gap_handle *h, const gap_atoms *atoms, const gap_sparse *sp,
                                const double *c, gap_precision prec, const double *g_e,
                                double *d_desc, double *d_c, double *d_X);

/* Forces from descriptor gradients by the chain rule (Sec. "Theory"):
 *   forces[j][alpha] = - sum_{(i,k): j(i,k)=j} J[(i,k)][alpha] . dEdd[i]
 * dEdd [n_atoms][D] FP64 row-major (ld = D); forces [n_atoms][3] FP64.
 * Deterministic: per-pair contributions are summed per target in pair order. */
gap_status gap_forces(gap_handle *h, const gap_atoms *atoms, const double *dEdd, double *forces);

/* The split step of the BF16X3 form on its own (the BF16X3 calls apply the
 * same split to their operands inside; reading of the split-BF16 contraction):
 * every value x of the row-major rows x cols array `x` (f32 or f64, leading
 * dimension ld, ld % 4 == 0, 32-byte aligned) becomes
 *   hi = bf16(fp32(x)),  lo = bf16(fp32(x) - hi)     (each rounding to nearest even)
 * written as raw bf16 bits to hi and lo [rows][ldp] (16-byte aligned), with
 * ldp = cols rounded up to a multiple of 32 and the padding zero.  hi_t / lo_t
 * (FP64 input only; both or neither) also receive the transposed halves
 * [cols][rows rounded up to 32], zero padded: the layout the library keeps of
 * the sparse points for W X.  FP64 input with hi_t runs the sparse-point split
 * kernel, every other call the Jacobian split kernel.  Asynchronous. */
gap_status gap_split_bf16x3(gap_handle *h, const void *x, gap_dtype dt, int64_t rows, int64_t cols,
                            int64_t ld, uint16_t *hi, uint16_t *lo, uint16_t *hi_t, uint16_t *lo_t);

/* gap_forces without any device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results as gap_forces;
 * its pair transposition and per-pair products live in a static device array
 * of 64 MiB (one per GPU, held until the process ends) instead of the handle's
 * workspace.  It needs 16 n_atoms + 32 n_pairs bytes plus about 10 KB
 * (and 8 n_atoms round4(D) more when dEdd is not 32-byte aligned or D % 4 != 0),
 * e.g. up to about 2 million pairs; larger inputs return GAP_E_INVALID before
 * anything is enqueued.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (several handles or streams) race and must be ordered by
 * the caller.  Asynchronous. */
gap_status gap_forces_noalloc(gap_handle *h, const gap_atoms *atoms, const double *dEdd,
                              double *forces);

/* Stage timing (profiling aid, off by default).  When enabled, the library
 * records HIP events on the handle's stream around each stage it enqueues;
 * gap_timing_read waits for them and returns the accumulated milliseconds and
 * the number of intervals per stage (arrays of gap_timing_count() entries, host),
 * optionally resetting the accumulators.  Stage names: gap_timing_name(i). */
gap_status gap_timing(gap_handle *h, int enable);
gap_status gap_timing_read(gap_handle *h, double *ms, int64_t *count, int reset);
const char *gap_timing_name(int i);
int gap_timing_count(void);

#ifdef __cplusplus
}
#endif

#endif /* GAP_H */
