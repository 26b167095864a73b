// Host-side launchers of the gfx950 kernels (implemented in the .hip files).
// Every launcher only enqueues work on `st`; argument validation is done by
// the C ABI layer before these are called.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <tuple>
#include <vector>

// Device status word bits (accumulated with atomicOr, read by synchronising calls).
#define GAP_DEVERR_INDEX 1   // a pair target or pointer outside its range
#define GAP_DEVERR_NOT_PD 2  // non-positive or non-finite Cholesky pivot
#define GAP_DEVERR_RANK 4    // zero or non-finite diagonal of R
#define GAP_DEVERR_SYNC 8    // a grid barrier timed out (cooperative launch not co-resident)

namespace gapk {

// Optional per-stage timing with HIP events recorded on the launch stream
// (a profiling aid: off unless the caller enables it on the handle).
enum TimerCat {
  TM_PAIRS = 0, TM_KMM, TM_ENERGY, TM_FORCE, TM_CHOL, TM_QR_PANEL, TM_QR_UPDATE, TM_TRSV,
  TM_PREDICT, TM_BACKWARD, TM_REFINE, TM_SPLIT, TM_COUNT
};
struct Timer {
  bool on = false;
  hipStream_t st = nullptr;
  hipEvent_t open[TM_COUNT] = {};
  std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> pending;
  void begin(int c) {
    if (!on) return;
    if (hipEventCreate(&open[c]) != hipSuccess) return;
    (void)hipEventRecord(open[c], st);
  }
  void end(int c) {
    if (!on || !open[c]) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, st);
    pending.emplace_back(c, open[c], e);
    open[c] = nullptr;
  }
  // Accumulate finished intervals into ms[c], count[c] (waits for the events).
  void collect(double* ms, int64_t* count) {
    for (auto& p : pending) {
      float t = 0.f;
      (void)hipEventSynchronize(std::get<2>(p));
      if (hipEventElapsedTime(&t, std::get<1>(p), std::get<2>(p)) == hipSuccess) {
        ms[std::get<0>(p)] += t;
        count[std::get<0>(p)] += 1;
      }
      (void)hipEventDestroy(std::get<1>(p));
      (void)hipEventDestroy(std::get<2>(p));
    }
    pending.clear();
  }
};

// ---- pairs.hip ------------------------------------------------------------
// tgt_ptr/tgt_pair (target-major pair view), pair_src, and the targets sorted
// by decreasing in-degree (order).  scratch_i32 needs n_atoms + 2048 ints.
void pair_transpose(const int64_t* pair_ptr, const int32_t* pair_j, int64_t n_atoms,
                    int64_t n_pairs, int64_t* tgt_ptr, int32_t* tgt_pair, int32_t* pair_src,
                    int32_t* order, int32_t* scratch_i32, int* dev_err, hipStream_t st);
// Configuration index of each atom (atom_cfg[i] = c for cfg_ptr[c] <= i < cfg_ptr[c+1]).
void atom_config(const int64_t* cfg_ptr, int64_t n_cfg, int64_t n_atoms, int32_t* atom_cfg,
                 hipStream_t st);

// ---- dense_f64.hip --------------------------------------------------------
void kmm_f64(const double* X, int64_t ldx, int64_t M, int64_t D, int zeta, double delta,
             double* K, int64_t ldk, hipStream_t st);
// Energy rows K[c][m] (col-major, ldk) and S[i][m] = delta^2 zeta p^(zeta-1) (row-major, ldS).
void energy_rows_f64(const void* desc, bool desc_f32, int64_t ldd, const int64_t* cfg_ptr,
                     int64_t n_cfg, int64_t n_atoms, const double* X, int64_t ldx, int64_t M,
                     int64_t D, int zeta, double delta, double* K, int64_t ldk, double* S,
                     int64_t ldS, hipStream_t st,
                     const int32_t* species = nullptr, int32_t zsel = 0);
// P-stage of predict / backward.  For rows i of desc:
//   mode 0 (forward):  W[i][m] = delta^2 zeta c_m p^(zeta-1)       (if W)
//                      e_atom[i] = sum_m c_m delta^2 p^zeta         (if e_atom)
//   mode 1 (backward): W[i][m] = g_e[i] delta^2 zeta c_m p^(zeta-1) (if W)
//                      dc_part[rb][m] = sum_{i in row block rb} g_e[i] delta^2 p^zeta
//   mode 2 (residual): W[i][m] = g_e[i] delta^2 p^zeta + delta^2 zeta p^(zeta-1) q_im
//                      where q = H X^T with H [n][ldh] (rows of h_i); only dc_part is written
//                      (column partial sums of W over the row block)
//   mode 3 (residual, force part with a stored S): dc_part = column partial sums of
//                      -S[i][m] q_im, q = H X^T (desc unused)
// Column groups of the LDS-staged P-stage; e_part (for e_atom in mode 0) holds
// pstage_groups(M) x n doubles.
int64_t pstage_groups(int64_t M);
void pstage_f64(int mode, const void* desc, bool desc_f32, int64_t ldd, int64_t n,
                const double* X, int64_t ldx, int64_t M, int64_t D, int zeta, double delta,
                const double* c, const double* g_e, const double* H, int64_t ldh, double* W,
                int64_t ldw, double* e_atom, double* dc_part, hipStream_t st,
                const double* Sx = nullptr, int64_t ldsx = 0, double* e_part = nullptr);
int64_t pstage_row_blocks(int64_t n);
// out[i][j] = scale_i * sum_k W[i][k] X[k][j]   (n x D, row-major ldo); scale = 1 if row_scale null
// Two-body SE descriptor: rows (energies, then 3 per atom) of the pair-distance
// kernel, its K_MM, and prediction (per-pair terms in ep / gp, n_pairs each).
void se2b_rows_f64(const double* pair_r, const int64_t* cfg_ptr, int64_t n_cfg,
                   const int64_t* pair_ptr, const int64_t* tgt_ptr, const int32_t* tgt_pair,
                   int64_t n_atoms, int64_t n_pairs, const double* x, int64_t M, double delta,
                   double theta, double r_cut, double width, double* K, int64_t ldk,
                   hipStream_t st);
void se2b_kmm_f64(const double* x, int64_t M, double delta, double theta, double r_cut,
                  double width, double* K, int64_t ldk, hipStream_t st);
void se2b_predict_f64(const double* pair_r, const int64_t* cfg_ptr, int64_t n_cfg,
                      const int64_t* pair_ptr, const int64_t* tgt_ptr, const int32_t* tgt_pair,
                      int64_t n_atoms, int64_t n_pairs, const double* x, const double* c,
                      int64_t M, double delta, double theta, double r_cut, double width,
                      double* ep, double* gp, double* e_cfg, double* forces, hipStream_t st);
// Virial rows: K[(9 c + 3 alpha + beta), m] = - sum_{p in c} r[p][alpha] S[src(p)][m] (J[p][beta] . x_m).
void virial_rows_f64(const void* jac, bool jac_f32, int64_t ldj, int64_t D, const double* X,
                     int64_t ldx, int64_t M, const double* S, int64_t ldS, const int64_t* cfg_ptr,
                     int64_t n_cfg, const int64_t* pair_ptr, const int32_t* pair_src,
                     const double* pair_r, int64_t n_atoms, int64_t n_pairs, double* K,
                     int64_t ldk, hipStream_t st);
// Local-property rows: K[r][m] = delta^2 (d_{atom_idx[r]} . x_m)^zeta (atom_idx NULL:
// atom r), column-major, or row-major [n_local][ldk] with zero row padding.
void local_rows_f64(const void* desc, bool desc_f32, int64_t ldd, int64_t n_atoms,
                    const int32_t* atom_idx, int64_t n_local, const double* X, int64_t ldx,
                    int64_t M, int64_t D, int zeta, double delta, double* K, int64_t ldk,
                    int* dev_err, hipStream_t st, bool row_major = false);
void gemm_wx_f64(const double* W, int64_t ldw, int64_t n, int64_t M, const double* X,
                 int64_t ldx, int64_t D, double* out, int64_t ldo, hipStream_t st);
// dc_part[rg][m] = -sum_{i in row group rg} S[i][m] (H_i . x_m), column-stationary;
// returns false (nothing launched) when the shape is outside its limits
// (D <= 256, ldS and ldh multiples of 4).  Groups: resid_colsum_groups(n, M).
int64_t resid_colsum_groups(int64_t n, int64_t M);
bool resid_colsum_f64(const double* H, int64_t ldh, int64_t n, int64_t D, const double* X,
                      int64_t ldx, int64_t M, const double* S, int64_t ldS, double* dc_part,
                      hipStream_t st);
// out = (W diag(cs)) X   (cs: [M], any alignment)
void gemm_wx_scaled_f64(const double* W, int64_t ldw, int64_t n, int64_t M, const double* cs,
                        const double* X, int64_t ldx, int64_t D, double* out, int64_t ldo,
                        hipStream_t st);
// y = A x (column-major rows x cols);  y += A^T x
void gemv_cm_f64(const double* A, int64_t lda, int64_t rows, int64_t cols, const double* x,
                 double* y, hipStream_t st);
void gemvt_cm_add_f64(const double* A, int64_t lda, int64_t rows, int64_t cols, const double* x,
                      double* y, hipStream_t st);
// out[m][j] = sum_i W[i][m] desc[i][j]        (M x D, row-major ldo)
void gemm_wtd_f64(const double* W, int64_t ldw, int64_t n, int64_t M, const void* desc,
                  bool desc_f32, int64_t ldd, int64_t D, double* out, int64_t ldo,
                  hipStream_t st);
// dst[i][0:D] = src[i][0:D]
void copy_rows_f64(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n, int64_t D,
                   hipStream_t st);
// out[m] = sum_rb part[rb][m]
void reduce_rows_f64(const double* part, int64_t nparts, int64_t M, double* out, hipStream_t st);
// e_cfg[c] = sum_{i in c} e_atom[i]
// e_cfg[c] = sum_{i in c} (d_i . g_i) / zeta (energies from descriptor gradients).
void cfg_energy_from_grad(const void* desc, bool desc_f32, int64_t ldd, const double* g,
                          int64_t ldg, const int64_t* cfg_ptr, int64_t n_cfg, int64_t n, int64_t D,
                          int zeta, double* out, hipStream_t st);
// H[i] -= (v[c(i)] / zeta) d_i for every atom i of configuration c.
void sub_cfg_desc(double* H, int64_t ldh, const void* desc, bool desc_f32, int64_t ldd,
                  const double* v, const int64_t* cfg_ptr, int64_t n_cfg, int64_t n, int64_t D,
                  int zeta, hipStream_t st);
// Zero e_atom[i] and W row i (ldw doubles) of every atom i with species[i] != zsel.
void mask_species_rows(const int32_t* species, int32_t zsel, int64_t n, double* e_atom, double* W,
                       int64_t ldw, hipStream_t st, float* W32 = nullptr);
void segment_sum_f64(const double* e_atom, const int64_t* cfg_ptr, int64_t n_cfg, int64_t n,
                     double* e_cfg, hipStream_t st);

// ---- force_f64.hip --------------------------------------------------------
void force_rows_f64(const void* jac, bool jac_f32, int64_t ldj, int64_t D, const double* X,
                    int64_t ldx, int64_t M, const double* S, int64_t ldS, const int64_t* tgt_ptr,
                    const int32_t* tgt_pair, const int32_t* pair_src, const int32_t* order,
                    int64_t n_atoms, int64_t n_pairs, int64_t row0, double* K, int64_t ldk,
                    hipStream_t st);
// f_pair[p][alpha] = J[p][alpha] . g[src(p)], then forces[j][alpha] = -sum_{p -> j} f_pair[p][alpha]
void forces_f64(const void* jac, bool jac_f32, int64_t ldj, int64_t D, const double* g,
                int64_t ldg, const int32_t* pair_src, int64_t n_atoms, int64_t n_pairs,
                const int64_t* tgt_ptr, const int32_t* tgt_pair, double* f_pair, double* forces,
                hipStream_t st);
// h[i][:] = sum_k sum_alpha v[j(i,k)][alpha] J[(i,k)][alpha][:]  (n_atoms x D, ld = ldh)
void jac_transpose_apply_f64(const void* jac, bool jac_f32, int64_t ldj, int64_t D,
                             const int64_t* pair_ptr, const int32_t* pair_j, int64_t n_atoms,
                             int64_t n_pairs, const double* v, double* h, int64_t ldh,
                             hipStream_t st);

// ---- mixed.hip (split-BF16, BF16x3) ---------------------------------------
// Row length of split arrays: n rounded up to a multiple of 32 (zero padded).
int64_t split_ld(int64_t n);
// X -> hi/lo halves [M][split_ld(D)]; optionally also the transposed halves
// [D][split_ld(M)] (Xth/Xtl may be null).
void split_x_bf16(const double* X, int64_t ldx, int64_t M, int64_t D, __bf16* Xh, __bf16* Xl,
                  __bf16* Xth, __bf16* Xtl, hipStream_t st);
void energy_rows_bf16x3(const void* desc, bool desc_f32, int64_t ldd, const int64_t* cfg_ptr,
                        int64_t n_cfg, int64_t n_atoms, const __bf16* Xh, const __bf16* Xl,
                        int64_t M, int64_t D, int zeta, double delta, double* K, int64_t ldk,
                        float* S, int64_t ldS, hipStream_t st,
                        const int32_t* species = nullptr, int32_t zsel = 0);
void force_rows_bf16x3(const void* jac, bool jac_f32, int64_t ldj, int64_t D, const __bf16* Xh,
                       const __bf16* Xl, int64_t M, const float* S, int64_t ldS,
                       const int64_t* tgt_ptr, const int32_t* tgt_pair, const int32_t* pair_src,
                       const int32_t* order, int64_t n_atoms, int64_t n_pairs, int64_t row0,
                       double* K, int64_t ldk, hipStream_t st);
// J -> hi/lo halves [3 n_pairs][split_ld(D)] each.
void split_j_bf16(const void* jac, bool jac_f32, int64_t ldj, int64_t n_pairs, int64_t D,
                  __bf16* Jh, __bf16* Jl, hipStream_t st);
// Any row-major rows x D array (ld % 4 == 0) -> hi/lo halves [rows][split_ld(D)].
void split_rows_bf16(const void* x, bool x_f32, int64_t ld, int64_t rows, int64_t D,
                     __bf16* hi, __bf16* lo, hipStream_t st);
// Force rows from pre-split Jacobians (returns false when D is too large for it).
bool force_rows_bf16x3_split(const __bf16* Jh, const __bf16* Jl, int64_t D, const __bf16* Xh,
                             const __bf16* Xl, int64_t M, const float* S, int64_t ldS,
                             const int64_t* tgt_ptr, const int32_t* tgt_pair,
                             const int32_t* pair_src, const int32_t* order, int64_t n_atoms,
                             int64_t n_pairs, int64_t row0, double* K, int64_t ldk,
                             hipStream_t st);
// ---- gemm_b3.hip (tiled BF16x3 GEMM for predict and backward) --------------
// Column / row blocks of its 128 x 128 tiles (sizes of the e / dc partials).
int64_t gemm_b3_col_blocks(int64_t n_b);
int64_t gemm_b3_row_blocks(int64_t n_a);
// P-stage: mode 0 e_part[cb][i] (cb < gemm_b3_col_blocks(M)) and W (FP32 [n][ldw]);
// mode 1 dc_part[rb][m] (rb < gemm_b3_row_blocks(n)) and W.
// X comes split (split_x_bf16's row halves, [M][split_ld(D)]).
void pstage_b3t(int mode, const void* desc, bool desc_f32, int64_t ldd, int64_t n,
                const __bf16* Xh, const __bf16* Xl, int64_t M, int64_t D, int zeta,
                double delta, const double* c, const double* g_e, float* W, int64_t ldw,
                double* e_part, double* dc_part, hipStream_t st);
// out[i][d] = sum_m W[i][m] X[m][d] from FP32 W and the split transposed X halves.
void gemm_b3_wx(const float* W, int64_t ldw, int64_t n, int64_t M, const __bf16* Xth,
                const __bf16* Xtl, int64_t D, double* out, int64_t ldo, hipStream_t st);
// out[m][d] = sum_i W[i][m] desc[i][d] (W FP32 [n][ldw]) with nz split-K partials
// in part [nz][M][D].
void gemm_b3_wtd(const float* W, int64_t ldw, int64_t M, int64_t n, const void* desc,
                 bool desc_f32, int64_t ldd, int64_t D, double* part, int nz, double* out,
                 int64_t ldo, hipStream_t st);
// out[i][j] = sum_z part[z * stride + i * cols + j].
void sum_parts_f64(const double* part, int64_t nz, int64_t stride, double* out, int64_t rows,
                   int64_t ldo, int64_t cols, hipStream_t st);
// ---- linalg.hip -----------------------------------------------------------
// A[r][0:M] *= 1/sigma_r, A[r][M] = y_r/sigma_r for r < n_rows.
void scale_rows(double* A, int64_t ld, int64_t n_rows, int64_t M, const double* y,
                const double* sigma, hipStream_t st);
// Rows n_rows .. n_rows+M-1 of A: U = L^T from the lower factor L (col-major
// ldl), and 0 in column M.
void stack_u(double* A, int64_t ld, int64_t n_rows, int64_t M, const double* L, int64_t ldl,
             hipStream_t st);
// In-place lower Cholesky of the M x M col-major matrix Lw (ld = ldl) after adding
// jitter to its diagonal; the strict upper part is left untouched.
void cholesky_lower(double* Lw, int64_t ldl, int64_t M, double jitter, const double* Kmm,
                    int64_t ldk, int* dev_err, hipStream_t st);
struct QrWork {
  double* part;       // split-K partials
  int64_t part_elems;
  double* W;          // nb x (n+1) reduced V^T C
  double* Wt;         // T^T W
  double* T;          // nb x nb
  double* colstate;   // per column: tau, beta, scale, then tw[nb]
  double* red;        // panel reduction partials
  double* tau;        // tau of every reflector [n]
  unsigned int* counter;
  unsigned int* flags;  // per-block completion flags of the multi-block triangular solves
};
size_t qr_workspace_bytes(int64_t m, int64_t n);
void qr_bind_workspace(void* base, int64_t m, int64_t n, QrWork* w);
// Householder QR of the m x ncols col-major A (ncols = n + 1 with b last); R in the
// upper triangle of the first n columns, Q^T b in column n.
void qr_factor(double* A, int64_t ld, int64_t m, int64_t ncols, int64_t n, QrWork* w,
               hipStream_t st, int* dev_err, Timer* tm = nullptr);
// x = R^-1 z (R upper n x n col-major in A, z = A[0:n][n]); records min/max |R_kk|
// into rd[0..1] (device) and flags zero/non-finite pivots.
// flags (QrWork::flags, may be NULL) enables the multi-block solve; x must not
// alias z when flags are given.
void back_substitute(const double* A, int64_t ld, int64_t n, const double* z, double* x,
                     double* rd, int* dev_err, hipStream_t st, unsigned int* flags = nullptr);
// Solve R^T y = x (forward) then R x = y (backward), result in x; with flags
// and an n-element scratch tmp, both solves use the multi-block kernel.
void seminormal_solve(const double* A, int64_t ld, int64_t n, double* x, hipStream_t st,
                      unsigned int* flags = nullptr, double* tmp = nullptr,
                      int* dev_err = nullptr);
// r_top[r] = (y_r - kc_r) / sigma_r
void residual_top(const double* y, const double* sigma, const double* kc, int64_t n_rows,
                  double* r_top, hipStream_t st);
// r_bot = -U c  (U = L^T, L lower M x M col-major)
void residual_bot(const double* L, int64_t ldl, int64_t M, const double* c, double* r_bot,
                  hipStream_t st);
// g[m] += (U^T r_bot)[m]  (U = L^T)
void add_ut_r(const double* L, int64_t ldl, int64_t M, const double* r_bot, double* g,
              hipStream_t st);
// v[r] = r_top[r] / sigma_r (weights for K^T)
void div_sigma(const double* r_top, const double* sigma, int64_t n, double* v, hipStream_t st);
void fill_f64(double* p, int64_t n, double v, hipStream_t st);
void axpy_f64(int64_t n, double a, const double* x, double* y, hipStream_t st);
void norm2_f64(const double* x, int64_t n, double* out, hipStream_t st);
// out[0] += x . x
void sumsq_add_f64(const double* x, int64_t n, double* out, hipStream_t st);
// Y = R^-1 (R upper n x n col-major) as a row-major Y[i * ldy + c], zero below
// the diagonal; one workgroup per column.
void trinv_upper(const double* R, int64_t ld, int64_t n, double* Y, int64_t ldy, int* dev_err,
                 hipStream_t st);
// var[i] = base + sign * ||Z[i][0:m]||^2 with base var[i] (init 0), delta^2 (d_i . d_i)^zeta
// (init 1) or 0 (init 2).
void var_rows(const double* Z, int64_t ldz, int64_t n, int64_t m, double sign, const void* desc,
              bool desc_f32, int64_t ldd, int64_t D, int zeta, double delta, int init,
              double* var, hipStream_t st);
// Descriptors as FP64 rows [n][ldo], zero row padding.
void desc_f64(const void* desc, bool desc_f32, int64_t ldd, int64_t n, int64_t D, double* out,
              int64_t ldo, hipStream_t st);
// CUR selection: keys (leverage, or log(u) / leverage) sorted into decreasing
// order, ties by index; key and idx hold cur_pad(n) entries.
int64_t cur_pad(int64_t n);
void cur_select_sort(const double* lev, const double* u, int64_t n, double* key, int32_t* idx,
                     hipStream_t st);
// Streamed-fit state: clear rows (col, M] of columns [0, M) of T (and T[M][M]
// when zero_corner).
void fold_tidy(double* T, int64_t ld, int64_t M, bool zero_corner, hipStream_t st);
// Expand per-configuration weights to atoms: out[i] = v[cfg(i)]
void expand_cfg(const double* v, const int32_t* atom_cfg, int64_t n_atoms, double* out,
                hipStream_t st);

}  // namespace gapk
