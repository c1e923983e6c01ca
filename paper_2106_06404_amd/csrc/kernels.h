// Host-side launchers of the msdd kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

typedef int64_t i64;
typedef int32_t i32;

// band.hip
void launch_neumann_assemble(hipStream_t s, i64 total_rows, const i32* row_sub, const i64* voff,
                             const i32* bw, const i64* boff, const i64* inc_ptr,
                             const i32* inc_slot, const i32* inc_a, const i32* slot_elem,
                             const i32* slot_loc, int k, const double* elem_mat, double* band,
                             int ell_w, const i32* ell_col, double* ell_val, int* status,
                             const i32* elem_ov = nullptr, double* band2 = nullptr,
                             double* ell_val2 = nullptr);
void launch_dirichlet_extract(hipStream_t s, i64 total_rows, const i32* drow_sub,
                              const i64* doff, const i32* nd, const i32* bd, const i64* dboff,
                              const i32* dglob, const i64* rowptr, const i32* col,
                              const double* val, double* band, int* status);
template <typename T>
void launch_band_cholesky(hipStream_t s, int nsubs, const i32* subs, int bmax, const i32* n_arr,
                          const i32* b_arr, const i64* src_off, const double* src,
                          const i64* dv_off, const double* dv, double sigma, const i64* dst_off,
                          T* Lc, T* Lr, int* status, const double* src2 = nullptr);
// Cholesky factor (column layout) -> LDL^T factor in row layout F and, in place,
// in column layout Lc (both with 1/D on the diagonal slot).
// band_blocked.hip: blocked solves with per-block inverses (half-bandwidth <= 64)
int64_t band_block_doubles(int n);  // storage of one subdomain's blocked factor
void launch_band_block_build(hipStream_t s, int nsubs, int nmax, int bmax, const i32* n_arr,
                             const i32* b_arr, const i64* l_off, const double* Fr,
                             const i64* blk_off, double* out);
void launch_band_solve_blk4(hipStream_t s, int nsubs, const i32* subs, int nmax,
                            const i32* n_arr, const i32* b_arr, const i64* blk_off,
                            const double* LB, const i64* v_off, int K, const double* W,
                            double* Y, const int* active);
void launch_band_solve_blk(hipStream_t s, int nsubs, const i32* subs, const i32* n_arr,
                           const i32* b_arr, const i64* blk_off, const double* LB,
                           const i64* v_off, int K, const double* W, double* Y,
                           const int* active);
template <typename T>
void launch_band_to_ldl(hipStream_t s, int nsubs, int nmax, int bmax, const i32* n_arr,
                        const i32* b_arr, const i64* off, T* Lc, T* F);
void launch_band_scale(hipStream_t s, int nsubs, int nmax, int bmax, const i32* n_arr,
                       const i32* b_arr, const i64* off, const i64* doff, double* B, double* sc,
                       int* status);
size_t band_cholesky_lds(int bmax, int elem_size);
// Y = A^{-1} W for K columns per subdomain with the LDL^T factor (Fc, Fr layouts).
template <typename T, typename V>
void launch_band_solve_multi(hipStream_t s, int nsubs, const i32* subs, int nmax,
                             const i32* n_arr, const i32* b_arr, const i64* l_off, const T* Fc,
                             const T* Fr, const i64* v_off, int K, const V* W, V* Y,
                             const int* active, int bmax, int variant = 0);

// eig.hip
void launch_eig_init(hipStream_t s, i64 total_rows, const i32* row_sub, const i64* voff,
                     const i32* nb, const i64* kvoff, int K, const double* dv, double* X,
                     unsigned long long seed, const i32* seed_id);
// Z = b Y with the columns staged in LDS per 256-row tile (band halo included); false
// (nothing launched) when the half-bandwidth makes the tile too large.
bool launch_bapply_tile(hipStream_t s, int P, int nmax, int bmax, const i64* voff, const i32* nb,
                        const i32* bw, const i64* kvoff, int K, const double* dv, int ell_w,
                        const i32* ell_col, const double* ell_val, const double* Y, double* Z,
                        const int* active);
void launch_bapply_ell(hipStream_t s, i64 total_rows, const i32* row_sub, const i64* voff,
                       const i32* nb, const i64* kvoff, int K, const double* dv, int ell_w,
                       const i32* ell_col, const double* ell_val, const double* Y, double* Z,
                       const int* active);
// Gram matrices as nsplit partial sums over row splits (GS, GB: P x nsplit x K x K)
void launch_gram(hipStream_t s, int P, const i32* nb, const i64* kvoff, int K, const double* Y,
                 const double* W, const double* Z, double* GS, double* GB, const int* active,
                 int nsplit);
void launch_rayleigh_ritz(hipStream_t s, int P, int K, const double* GS, const double* GB,
                          double* C, double* nu, const int* active, int nsplit, double* gs_diag);
// Cholesky factorisation of one large SPD matrix A (n x n, column-major, overwritten by L
// with the upper triangle zeroed), Linv = L^{-1} and Inv = A^{-1} (full, symmetric), in
// 64 x 64 tiles over the whole device; status[0] is set to ST_NOTSPD on a non-positive
// pivot (left untouched otherwise).  Linv and Inv: n x n each.
void launch_blocked_spd_inverse(hipStream_t s, int n, double* A, double* Linv, double* Inv,
                                int* status);
// partial sums per column and row split written by the eigensolver's update kernel
constexpr int UPD_PARTS = 4;
void launch_eig_update(hipStream_t s, int P, const i32* nb, const i64* kvoff, int K,
                       const double* C, const double* nu, const double* Y, const double* Z,
                       double* X, double* BX, double* SX, double sigma, double eta, int nev_max,
                       double tol, int maxit, int* status, int* iters, int* mcount,
                       double* lam_out, double* res_out, int Kmax_allowed, const i32* rankb,
                       const double* normS, double* nu_prev, double* part, int nsplit,
                       const double* gs_diag, const int* inertia, int nev_fixed, double tol_e,
                       double* res_e_out, const double* SY = nullptr);
void launch_row_norm(hipStream_t s, int P, const i64* voff, int ell_w, const i32* ell_col,
                     const double* ell_val, const double* dv, double sigma, double* normS,
                     const double* ell_val2 = nullptr);
void launch_eig_finalize(hipStream_t s, int P, const i32* nb, const i64* voff, const i64* kvoff,
                         int K, const double* dv, const double* X, const double* nu,
                         const int* mcount, const i64* phi_off, double* Phi, const i32* nd,
                         const i64* doff, const i32* dpos, const i64* phid_off, double* PhiD);

// coarse.hip
void launch_patch_gather(hipStream_t s, int np, const i64* pdof_ptr, const i32* pM,
                         const i64* mem_ptr, const i32* mem_sub, const i32* mem_col,
                         const i64* ploc_off, const i32* ploc, const i32* nb, const i32* msub,
                         const i64* phi_off, const double* Phi, const i64* vpoff, double* Vp);
void launch_patch_av(hipStream_t s, i64 total_rows, const i32* row_patch, const i64* pdof_ptr,
                     const i32* pM, const i64* inc_ptr, const i32* inc_slot, const i32* inc_a,
                     const i32* slot_elem, const i32* slot_loc, int k, const double* elem_mat,
                     const i64* vpoff, const double* Vp, double* Up);
void launch_patch_gram(hipStream_t s, int np, const i64* pdof_ptr, const i32* pM,
                       const i64* vpoff, const double* Vp, const double* Up, const i64* pmoff,
                       double* Pm);
void launch_patch_project(hipStream_t s, int nq, const i64* ch_ptr, const i32* ch_patch,
                          const i32* cM, const i64* cmoff, const double* Pc,
                          const i64* cmem_ptr, const i32* cmem_pslot, const i32* cmem_ownbase,
                          const i32* cmem_m, const i32* cmem_col, const i64* pmem_ptr,
                          const i32* pmem_sub, const i32* pmem_col, const i32* mpar,
                          const i32* nown, const i64* yoff, const double* Y, const i32* pMout,
                          const i64* poutoff, double* Pout, const i64* wsoff, double* Wsc);
void launch_coarse_assemble(hipStream_t s, int nt, const i64* tp_ptr, const i32* tp_patch,
                            const i64* tp_map_off, const i32* tp_map, const i32* pM,
                            const i64* pmoff, const double* Pm, const i32* ng_arr,
                            const i64* aoff, double* Aout);
void launch_dense_cholesky(hipStream_t s, int nt, int nmax, const i64* off, const i32* n_arr,
                           double* A, int* status);
// doubles of eigenvalues and eigensolver workspace of one coarse GEVP target of size ng
// (kept in its scratch when they do not fit in LDS)
int64_t coarse_gevp_vec_doubles(int ng);
void launch_coarse_gevp(hipStream_t s, int nt, const i32* ng_arr, const i32* no_arr,
                        const i64* aoff, double* Abar, const i64* loff, double* Lo,
                        const i64* soff, double* scratch, double eta, int nev_max,
                        double eps_reg, double* lam_out, const i64* lamoff, int* m_out,
                        int* status, int* rank_out, int* sweeps_out, int ng_max);
void launch_dense_to_layouts(hipStream_t s, int nt, const i64* off, const i32* n_arr,
                             const double* L, double* R, double* C);
void launch_spd_inverse(hipStream_t s, int nt, int nmax, const i64* off, const i32* n_arr,
                        const double* L, double* Linv, double* Inv);
void launch_coarse_collect(hipStream_t s, int nt, const i32* ng_arr, const i32* no_arr,
                           const i64* soff, const double* scratch, const int* m_arr,
                           const i64* yoff, double* Y);

// abar Y in difference form for the eigensolver with the single-precision factor
// (eig32.hip): rs = compensated row sums of the Neumann matrices (ELL), then
// T = abar Y row by row as sum_j a_rj (y_j - y_r) + rs_r y_r over the running subdomains
void launch_abar_rowsum(hipStream_t s, i64 total_rows, int ell_w, const i32* ell_col,
                        const double* ell_val, double* rs);
void launch_abar_diff(hipStream_t s, i64 total_rows, const i32* row_sub, const i64* voff,
                      const i32* nb, const i64* kvoff, int K, int ell_w, const i32* ell_col,
                      const double* ell_val, const double* rs, const double* Y, double* T,
                      const int* active);
// pcg.hip
// segmented PCG (see pcg.hip): per-segment state fields and reduction rules
enum { PCG_RZ = 0, PCG_PQ, PCG_RR, PCG_ALPHA, PCG_BETA, PCG_RR0, PCG_TOL2, PCG_SD };
enum { PCG_ACTIVE = 0, PCG_IT, PCG_ITERS, PCG_SI };
enum { PCG_RUNNING = 1, PCG_CONVERGED = 0, PCG_MAXIT = 2, PCG_BREAKDOWN = -1 };
enum { PCG_R_RR0 = 0, PCG_R_RZ0, PCG_R_PQ, PCG_R_RR, PCG_R_RZ };
void launch_spmv_chunk(hipStream_t s, int nch, int sg, const i64* ch_lo, const i64* ch_hi,
                       const i64* rowptr, const i32* col, const double* val, const double* p,
                       double* q, double* partial);
void launch_residual_chunk(hipStream_t s, int nch, const i64* ch_lo, const i64* ch_hi,
                           const double* b, const double* q, double* r, double* partial);
void launch_update_xr_chunk(hipStream_t s, int nch, const i64* ch_lo, const i64* ch_hi,
                            const i32* ch_seg, double* x, double* r, const double* p,
                            const double* q, const double* D, double* partial);
void launch_dot_chunk(hipStream_t s, int nch, const i64* ch_lo, const i64* ch_hi, const double* a,
                      const double* b, double* partial);
void launch_update_p_chunk(hipStream_t s, int nch, const i64* ch_lo, const i64* ch_hi,
                           const i32* ch_seg, const double* z, double* p, const double* D,
                           int first);
void launch_seg_reduce(hipStream_t s, int nseg, const i64* seg_ch, const double* partial,
                       double* D, int* I, int rule, double rtol, int maxit, double* hist);
// *flag = 1 if a row's columns leave its problem's dof range [pdp[t], pdp[t+1])
void launch_check_problem_coupling(hipStream_t s, i64 n, const i64* rowptr, const i32* col,
                                   const i64* pdp, int nprob, int* flag);
void launch_apply_fine_restrict(hipStream_t s, int P, int nd_max, const i32* nd, const i64* doff,
                                const i32* dglob, const i32* msub, const i64* moff,
                                const i64* phid_off, const double* PhiD, const double* r,
                                double* rc, double* u);
// u_i = A_i^{-1} u_i with the LDL^T factor (Fc column layout, Fr row layout) in double
// (fp32 = 0) or single precision (fp32 = 1; Fc, Fr are float and the factor is that of
// diag(scale) A_i diag(scale), scale given per Dirichlet dof).
void launch_apply_fine_solve(hipStream_t s, int P, int nd_max, int bd_max, const i32* nd,
                             const i32* bd, const i64* doff, const i64* dboff, const void* Fc,
                             const void* Fr, int fp32, const double* scale, double* u,
                             int variant = 0);
// eig.hip, the FP32-factor eigensolver: scaling of S, scaled band, block combinations
void launch_s_diag_scale(hipStream_t s, i64 total_rows, const i32* row_grp, const i64* voff,
                         const i64* boff, const i32* bw, const double* band, const double* gw,
                         double sigma, double* sc, int* status);
void launch_band_scale_sym(hipStream_t s, i64 total_rows, const i32* row_grp, const i64* voff,
                           const i64* boff, const i32* bw, const i32* nrows, const double* band,
                           const double* sc, double* out);
void launch_eig32_combine(hipStream_t s, int mode, int P, int nmax, const i32* nb,
                          const i64* voff, const i64* kvoff, int K, const double* P1,
                          const double* P2, const double* nu, const double* sc, double sigma,
                          double* out, const int* status);
// twist.hip: two-sided Dirichlet solves (top and bottom parts as two chains, explicit
// inverse of the separator's Schur complement)
void twist_split(int n, int b, int* nbt, int* nbb);  // nbt = 0: no split
size_t apply_fine_twist_lds(int nd_max, int bd_max, size_t elem, bool cinv_lds);
void launch_twist_extract(hipStream_t s, int P, int nB_max, int bd_max, const i32* nd,
                          const i32* bd, const i32* nbt, const i32* nbb, const i64* dboff,
                          const double* Dband, const i64* toff, double* Bt);
template <typename T>
void launch_twist_schur(hipStream_t s, int P, const i32* nd, const i32* bd, const i32* nbt,
                        const i32* nbb, const i64* dboff, const double* Dband, const T* Fr,
                        const i64* toff, const T* Gr, const i64* coff, T* Cinv, int* status);
bool launch_apply_fine_twist(hipStream_t s, int P, int nd_max, int bd_max, const i32* nd,
                             const i32* bd, const i64* doff, const i64* dboff, const void* Fc,
                             const void* Fr, const i32* nbt, const i32* nbb, const i64* toff,
                             const void* Gc, const void* Gr, const i64* coff, const void* Cinv,
                             int fp32, const double* scale, double* u);
void launch_apply_coarse_down(hipStream_t s, int P, int no_max, const i32* nown,
                              const i64* own_ptr, const i32* own_idx, const i64* loff,
                              const double* Inv, const i32* msub, const i64* yoff,
                              const double* Y, const i64* moff, const double* rl, double* zl,
                              double* rc);
void launch_apply_coarsest(hipStream_t s, int nt, int nmax, const i64* zoff, const i64* aoff,
                           const i32* n_arr, const double* Inv, const double* r0, double* z0);
void launch_apply_coarse_up(hipStream_t s, int P, const i32* nown, const i64* own_ptr,
                            const i32* own_idx, const i32* msub, const i64* yoff, const double* Y,
                            const i64* moff, const double* zc, double* zl);
// Number of eigenvalues below eta of each subdomain's pencil, by the inertia of
// abar + sigma D abar D (sigma = -eta); -1 where it could not be determined.
void launch_band_inertia(hipStream_t s, int nsubs, int bmax, const i32* n_arr, const i32* b_arr,
                         const i64* src_off, const double* src, const i64* dv_off,
                         const double* dv, double sigma, int* neg, const double* src2 = nullptr);
// gmres.hip: dense vector kernels of GMRES (x, y, V column-major with leading dimension n)
// h[c] = V(:, c) . w for c < k (partial sums per block, then a fixed-order reduction)
void launch_multi_dot(hipStream_t s, i64 n, int k, const double* V, const double* w,
                      double* partial, double* h);
// w -= V(:, 0:k) h
void launch_multi_axpy(hipStream_t s, i64 n, int k, const double* V, const double* h, double* w);
// y = V(:, 0:k) c   (acc: y += ...)
void launch_gemv_cols(hipStream_t s, i64 n, int k, const double* V, const double* c, double* y,
                      int acc);
// y = a * x, a read from the device scalar: a = ap[0] (inv 0), 1 / ap[0] (1), 1 / sqrt(ap[0]) (2)
void launch_scale_dev(hipStream_t s, i64 n, const double* ap, int inv, const double* x, double* y);
// y += a x (host scalar)
void launch_axpy(hipStream_t s, i64 n, double a, const double* x, double* y);
void launch_fill(hipStream_t s, i64 n, double v, double* y);
// number of blocks multi_dot uses for n rows (its partial array holds k * blocks)
int multi_dot_blocks(i64 n);

// Scratch array of msdd_solve_noalloc (pcg.hip): noalloc_scratch_init looks up its
// device address for `device` (which must be current), once; noalloc_scratch returns it
// (nullptr before the lookup).  Returns 0 or -1.
int noalloc_scratch_init(int device);
void* noalloc_scratch(int device);
void launch_apply_fine_up(hipStream_t s, i64 n, const i64* dinc_ptr, const i32* dinc_sub,
                          const i32* dinc_q, const i64* doff, const i32* msub, const i64* moff,
                          const i64* phid_off, const double* PhiD, const double* u,
                          const double* zc, double* z,
                          const double* w = nullptr, int acc = 0);
// the same gather over the PCG chunks (nch workgroups, rows ch_lo[c] .. ch_hi[c], at most
// 256 each), also writing partial[c] = the chunk's r.z as launch_dot_chunk computes it
void launch_apply_fine_up_dot(hipStream_t s, int nch, const i64* ch_lo, const i64* ch_hi,
                              const i64* dinc_ptr, const i32* dinc_sub, const i32* dinc_q,
                              const i64* doff, const i32* msub, const i64* moff,
                              const i64* phid_off, const double* PhiD, const double* u,
                              const double* zc, double* z, const double* r, double* partial);

// mlp.hip (warm-start network of the local eigensolver)
// C_z = opA(A) opB(B) over split z of K (row-major M x N partials); every split is
// non-empty, so at most `splits` are launched: the count launched is returned
int sgemm_splits(int K, int splits);
int launch_sgemm(hipStream_t s, int ta, int tb, int M, int N, int K, int splits, const float* A,
                 int lda, const float* B, int ldb, float* C);
void launch_splitk_epi(hipStream_t s, int M, int N, int splits, const float* part, const float* bias,
                       const float* h, int mode, float* out);
void launch_colsum(hipStream_t s, int M, int N, const float* D, float* g);
void launch_gather_rows(hipStream_t s, int B, int w, const int* idx, const float* src, float* dst);
void launch_proj_loss(hipStream_t s, int B, int V, int n_pos, int m_cap, const int* idx,
                      const float* y, const float* tgt, const float* mask, const int* cnt,
                      double ridge, float* dy, float* loss_b);
void launch_adam(hipStream_t s, i64 n, float* p, const float* g, float* m, float* v, float lr,
                 int step);
void launch_init_uniform(hipStream_t s, i64 lo, i64 hi, float a, unsigned long long seed, float* w);
void launch_to_bf16(hipStream_t s, int rows, int cols, int ldd, const float* src, int lds,
                    unsigned short* dst);
void launch_to_bf16_t(hipStream_t s, int rows, int cols, int ldd, const float* src, int lds,
                      unsigned short* dst);
void launch_hgemm(hipStream_t s, int M, int N, int Kp, const unsigned short* A, const unsigned short* Bt,
                  const float* bias, int relu, int out_bf16, void* C, int ldc);
void launch_eig_init_warm(hipStream_t s, i64 total_rows, const i32* row_sub, const i64* voff,
                          const i32* nb, const i64* kvoff, int K, const double* dv, double* X,
                          unsigned long long seed, const i32* seed_id, const int* warm,
                          const float* yw, int n_vec, int n_pos, const i32* pos);
void launch_warm_targets(hipStream_t s, int nsel, const int* sel, const i32* nb, const i64* voff,
                         const i64* kvoff, int K, const double* X, const int* mcount, int m_cap,
                         int n_pos, const i32* pos, float* tgt, float* mask, int* cnt);
