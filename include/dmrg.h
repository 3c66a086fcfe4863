/*
 * dmrg.h -- C ABI of the MI355X (gfx950) two-site ab initio DMRG sigma library.
 *
 * The library computes the hot path of two-site DMRG on the matrix product
 * state (MPS) of eq. (1) of the paper: the renormalised block operators of
 * the quantum-chemistry Hamiltonian (Method section; the "DMRG matrix and
 * tensor algebra" of the Hardware section) and the Davidson sigma step
 * sigma = H_eff psi on a two-site window.  Quantum numbers are U(1) x U(1):
 * particle number N and 2*Sz.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Orbitals 0..K-1 are the MPS sites in chain order; spin-orbital
 *   p = 2*orbital + spin (spin 0 = up, 1 = down).  The local basis of a site
 *   is |0>, |up>, |dn>, |updn> (indices 0..3) with |updn> = a+_up a+_dn |0>,
 *   carrying (N, 2Sz) = (0,0), (1,+1), (1,-1), (2,0).
 * - H = e_core + sum_{pq,s} h_pq a+_{ps} a_{qs}
 *       + 1/2 sum_{pqrs,st} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}
 *   with h symmetric (K*K, row-major) and (pq|rs) in chemists' notation
 *   (K^4, row-major, 8-fold symmetric).
 * - Bond b (0..K) lies left of site b.  Each bond holds sectors labelled by
 *   the (N, 2Sz) of the sites left of it, sorted ascending by (N, 2Sz);
 *   bond 0 is (0,0) with dim 1 and bond K is (N_total, 2Sz_total) with dim 1.
 * - Site tensor b: blocks (l, n) -> r with Q_l + Q_n = Q_r (l a sector of
 *   bond b, r of bond b+1), packed by ascending l then n, each block d_l x d_r
 *   row-major; absent r means absent block.  Sites left of the window are
 *   left-canonical, sites right of it right-canonical.
 * - psi of window (i, i+1) ("right-sector-major"): for every sector r of
 *   bond i+2 in ascending order, the rows (l, n1, n2) with
 *   Q_l + Q_n1 + Q_n2 = Q_r in ascending (l, n1, n2) order form one dense
 *   M_r x d_r row-major matrix (the rows of one (l, n1, n2) are d_l
 *   consecutive rows).  sigma uses the same layout.
 *
 * Ownership: the caller owns every buffer it passes; the library copies what
 * it keeps (integrals, MPS) and never frees caller memory.  The context owns
 * all derived device state until dmrg_destroy.
 *
 * Streams: device work of a context is ordered on the stream given to
 * dmrg_create (NULL = the null stream).  Device pointers passed to a call must
 * be valid on that stream.  Calls return after their device work is
 * enqueued; dmrg_sigma does not synchronise.
 *
 * Errors: every call returns a status; < 0 is an error and leaves the
 * caller's buffers untouched, > 0 a warning.  dmrg_last_error gives the
 * message.  Arguments are validated on the host before any device work.
 */
#ifndef DMRG_H
#define DMRG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dmrg_status;
#define DMRG_OK 0
#define DMRG_WARN_NOT_CONVERGED 1
#define DMRG_ERR_INVALID_ARG (-1)
#define DMRG_ERR_SHAPE (-2)
#define DMRG_ERR_HIP (-3)
#define DMRG_ERR_OOM (-4)
#define DMRG_ERR_NO_DEVICE (-5)
#define DMRG_ERR_UNIMPLEMENTED (-6)
#define DMRG_ERR_STATE (-7)

/* Arithmetic of the sigma contractions. */
#define DMRG_FP64 0   /* FP64 MFMA, FP64 accumulation */
#define DMRG_BF16 1   /* BF16 MFMA, FP32 accumulation, FP64 output */
#define DMRG_BF16X3 2 /* split-BF16 (hi*hi + hi*lo + lo*hi), FP32 accumulation */
#define DMRG_OZAKI 3  /* FP64 emulated on INT8 MFMA (Ozaki scheme; Hardware section):
                         each operand row scaled by a power of two and split into
                         kappa signed 8-bit digits (8 kappa - 1 bits, kappa from
                         DMRG_OZAKI_SLICES, default 6: 47 bits), the kappa (kappa+1)/2
                         leading digit products exact in INT32, combined in FP64 */

typedef struct dmrg_ctx_s* dmrg_ctx;

/* Active space and integrals (host pointers, read during the call). */
typedef struct {
  int32_t n_orb;   /* K */
  int32_t n_elec;  /* N, 0 <= N <= 2K */
  int32_t two_sz;  /* 2*Sz, |2Sz| <= min(N, 2K-N), same parity as N */
  int32_t pad;
  double e_core;   /* constant added to every energy */
  const double* h;   /* K*K */
  const double* eri; /* K^4, chemists' (pq|rs) */
} dmrg_problem;

/* U(1) block-sparse MPS (host pointers, copied during the call). */
typedef struct {
  int32_t n_sites;              /* K */
  int32_t window;               /* i: the two-site window is (i, i+1) */
  const int32_t* bond_offsets;  /* K+2 entries: sectors of bond b are [off[b], off[b+1]) */
  const int32_t* sector_n;
  const int32_t* sector_2sz;
  const int32_t* sector_dim;
  const double* const* site_data; /* K pointers; entries i and i+1 are ignored */
} dmrg_mps;

/* Creates a context on HIP device `device`; `stream` is a hipStream_t (may be
 * NULL).  Fails with DMRG_ERR_NO_DEVICE when no such device exists. */
dmrg_status dmrg_create(dmrg_ctx* out, int32_t device, void* stream);
dmrg_status dmrg_destroy(dmrg_ctx ctx);
/* Message of the last error of ctx (or of the calling thread when ctx is NULL). */
const char* dmrg_last_error(dmrg_ctx ctx);

/* Builds the renormalised operators for the window (site, site+1)
 * (Method section; White-Martin / Chan-Head-Gordon normal and complementary
 * operators): the left block of sites [0, site) and the right block of sites
 * [site+2, K).  problem / mps may be NULL to keep the ones already loaded
 * (a new one invalidates every cached block).  direction (+1 / -1 / 0) only
 * hints which cached blocks to keep.  precision_mask: bit p requests the
 * operator copies for precision p (bit 0 = FP64 is always built). */
dmrg_status dmrg_build_ops(dmrg_ctx ctx, const dmrg_problem* problem, const dmrg_mps* mps,
                           int32_t site, int32_t direction, uint32_t precision_mask);

/* Number of doubles of psi / sigma for the current window. */
dmrg_status dmrg_psi_size(dmrg_ctx ctx, int64_t* n);

/* sigma = H_eff psi for the current window (device pointers, length
 * dmrg_psi_size, layout in the header comment).  H_eff is the projection
 * P^T H P of H onto the window's MPS basis, without e_core. */
dmrg_status dmrg_sigma(dmrg_ctx ctx, const double* psi, double* sigma, int32_t precision);

typedef struct {
  double flops;          /* algorithmic FLOPs of one sigma (2*m*n*k over block GEMMs) */
  double hw_flops;       /* MFMA operations issued: flops, 3x flops for DMRG_BF16X3,
                            kappa (kappa + 1) / 2 x flops INT8 operations for DMRG_OZAKI */
  int64_t n_pairs;       /* operator pairs (left op, site matrix, right op) */
  int64_t n_right_ops;   /* distinct right operators contracted first */
  int64_t n_stage1_tiles, n_stage2_tiles, n_stage2_segments;
  int64_t workspace_bytes;
  int64_t operator_bytes; /* device bytes of the left + right block operators */
  int32_t n_chunks;
  int32_t pad;
  double flops_stage1;   /* psi x right operators */
  double flops_stage2;   /* left operators x stage-1 results */
  /* BF16 launch configuration per stage, chosen by the autotuner on the
   * first mixed-precision sigma of the window (until then the default):
   * tile shape (0: 128x64, 1: 64x64, 2: 64x128, 3: 128x128, 4: 128x128 with
   * three LDS stages, 5: 256x256 with eight waves (stage 2; stage 1 then
   * uses 4), 6: chosen per output problem, 7: 128x128 over the whole
   * 128-blocks of each output problem and 64-wide tiles over remainders of
   * at most 64 rows or columns) + 16 * tile grouping
   * (0: per output problem, 1: per operand-sharing key) + 256 * segment
   * order (1: sorted by operand) */
  int32_t bf_config_stage1, bf_config_stage2;
  double tune_ms;        /* time the autotuner took (0 if it did not run) */
  double flops_terms;    /* the per-term count: sum over (Hamiltonian term, psi block) of the
                            cheaper association order, min(2m'mn + 2m'nn', 2mnn' + 2m'mn') for
                            O_L (m' x m) psi (m x n) O_R^T (n x n'); beside `flops`, which counts
                            the GEMMs issued (stage 1 is shared by every term with the same right
                            operator and multiplies whole psi sectors) */
  double flops_stage1_used; /* stage-1 FLOPs of the rows that stage 2 reads */
} dmrg_sigma_info;
dmrg_status dmrg_sigma_get_info(dmrg_ctx ctx, int32_t precision, dmrg_sigma_info* out);

/* Graph replay of the sigma (batching of its launches): with enable = 1,
 * every sigma of the context (dmrg_sigma and the Davidson solver's) replays
 * a HIP graph holding all of its launches, captured on the first call per
 * precision and window; host work (binding the caller's buffers, BF16
 * preparation) stays outside the graph.  Results are identical to the
 * launches made one by one.  Default 0; kept across dmrg_build_ops.  Kernel
 * timing (dmrg_sigma_timing) bypasses the graphs while it is on. */
dmrg_status dmrg_sigma_graphs(dmrg_ctx ctx, int32_t enable);

/* Kernel timing of dmrg_sigma: HIP events recorded on the context stream
 * around every grouped-GEMM launch of a sigma (diagnostic; off by default).
 * mode 1 resets the totals and starts timing, 0 stops, -1 leaves it as is.
 * out (may be NULL) receives the totals of the calls timed so far; reading
 * them synchronises the stream.  Times are summed over calls. */
typedef struct {
  int32_t calls;              /* sigma calls timed */
  int32_t launches_stage1;    /* stage-1 launches (psi x right operators), summed */
  int32_t launches_stage2;    /* stage-2 launches (left operators x stage 1) */
  int32_t launches_pinned;    /* FP64 launches of the block-Hamiltonian pairs */
  double ms_stage1, ms_stage2, ms_pinned;
  double flops_stage1, flops_stage2, flops_pinned;  /* algorithmic FLOPs of one call */
  int32_t launches_convert;   /* operand conversion launches (DMRG_OZAKI: digit slicing of psi and of
                                 the stage-1 results) */
  int32_t pad;
  double ms_convert;
} dmrg_sigma_times;
dmrg_status dmrg_sigma_timing(dmrg_ctx ctx, int32_t mode, dmrg_sigma_times* out);

/* Davidson solve for the lowest eigenpair of H_eff at the current window
 * (Davidson 1975, diagonal preconditioner, thick restart to the Ritz vector;
 * the Numerical-procedure section's eigensolver tolerance is a residual
 * norm, here ||H_eff u - theta u||_2 with ||u||_2 = 1).  Sigma products run
 * through a precision ladder: stage s uses ladder[s] until the residual is
 * below ladder_tol[s], reaches 3x the floor its sigma error allows (relative
 * sigma error 4e-3 BF16, 3e-6 split-BF16x3, 1e-13 Ozaki, times |theta|) or
 * gains less than 10% in 10 iterations; then the subspace restarts from the
 * Ritz vector; the last stage must be DMRG_FP64 and runs to tol.  Orthogonalisation
 * and the subspace matrices are FP64.  energy_out = FP64 Rayleigh quotient
 * + e_core.  psi_inout: start vector in, normalised Ritz vector out.
 * Returns DMRG_WARN_NOT_CONVERGED (with the best vector and energy) when
 * max_iter corrections were not enough. */
typedef struct {
  int32_t max_iter;      /* correction vectors (default 100) */
  int32_t max_subspace;  /* 3..64 (default 24) */
  double tol;            /* default 1e-6 */
  int32_t n_ladder;      /* 1..4 */
  int32_t ladder[4];     /* DMRG_FP64 / DMRG_BF16 / DMRG_BF16X3 / DMRG_OZAKI per stage */
  double ladder_tol[4];  /* stage-end residuals (all stages but the last) */
  int32_t precondition;  /* 2: Olsen-corrected diag(H_eff) (recommended), 1: plain diag(H_eff), 0: none */
  int32_t restart;       /* Ritz vectors kept at a thick restart (default 6) */
  int32_t refine;        /* 1: when the ladder reaches its DMRG_FP64 stage from a reduced
                            precision, residual refinement (Jacobi-Davidson with inexact inner
                            solves): the FP64 stage keeps its subspace, FP64 sigma products
                            and Rayleigh-Ritz, but each correction t solves
                            (1 - u u^T)(H - theta)(1 - u u^T) t = -r (t orthogonal to u) for
                            the Ritz pair (theta, u) and its FP64 residual r, by
                            preconditioned conjugate gradients on the previous stage's
                            reduced-precision sigma to 1e-2 relative (at most 60 products,
                            each counted as an iteration).  0: off (default) */
} dmrg_davidson_opts;

typedef struct {
  double energy, residual, time_ms, sigma_ms;
  int32_t iterations, converged;
  int32_t n_sigma[4];    /* sigma products per precision (DMRG_FP64 .. DMRG_OZAKI) */
  int32_t n_history;     /* entries used below (<= 256) */
  double residual_history[256];
  int32_t stage_history[256];
} dmrg_davidson_stats;

dmrg_status dmrg_davidson(dmrg_ctx ctx, double* psi_inout, const dmrg_davidson_opts* opts,
                          double* energy_out, dmrg_davidson_stats* stats_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * sigma of dmrg_sigma (same kernels, same result) with its stage-1 workspace
 * in a fixed 64 MiB device array that the library holds per GPU until the
 * process ends.  The call itself allocates nothing: its descriptors are built
 * by dmrg_build_ops.  psi, sigma: device pointers as for dmrg_sigma.  A window
 * whose stage-1 workspace (one chunk) exceeds 64 MiB is refused with
 * DMRG_ERR_SHAPE; create the context with DMRG_WS_BUDGET_MB <= 64 to chunk
 * it below that.  Every context on a GPU shares that GPU's array, so calls
 * that overlap on one GPU (from several contexts or streams) race; calls
 * ordered on one stream do not.  Graph replay (dmrg_sigma_graphs) and kernel
 * timing do not apply.  Stream-ordered, no synchronisation (except when the
 * psi / sigma pointers differ from the previous call's). */
dmrg_status dmrg_sigma_noalloc(dmrg_ctx ctx, const double* psi, double* sigma);

/* Reverse mode of the sigma with respect to the integrals.  For window
 * vectors psi and sigma_bar (device, psi layout of the current window;
 * sigma_bar NULL means psi) and the current MPS, f = <sigma_bar, H_eff psi>
 * is linear in the integrals of the Hamiltonian (Method section: the ab initio
 * Hamiltonian with one- and two-electron integrals); its gradient is written
 * to dh (K*K) and deri (K^4), device pointers, same index order as the
 * integrals, overwritten:
 *   dh[p][q]         = sum_s <sigma_bar| a+_ps a_qs |psi>             (gamma_pq)
 *   deri[p][q][r][s] = 1/2 sum_{s,t} <sigma_bar| a+_ps a+_rt a_st a_qs |psi>
 * in the full-space states of the MPS with the window vectors in place.  With
 * sigma_bar = psi normalised these are dE/dh = gamma and dE/d(pq|rs) =
 * Gamma_pqrs / 2 at fixed MPS (every entry an independent input).  The
 * operator adjoints are carried back along both blocks, so the call rebuilds
 * both blocks once (FP64); it synchronises the stream before returning.
 * precision: DMRG_FP64 runs every adjoint contraction on FP64 MFMA;
 * DMRG_BF16X3 (the mixed variant) and DMRG_BF16 run them on the BF16 kernel
 * (split-BF16x3 or plain BF16 products, FP32 accumulation flushed into FP64),
 * the integral gradient being accumulated in FP64 either way. */
dmrg_status dmrg_sigma_backward(dmrg_ctx ctx, const double* psi, const double* sigma_bar,
                                double* dh, double* deri, int32_t precision);

/* Orbital gradient for orbital optimisation (DMRG-SCF), the consumer of
 * dmrg_sigma_backward.  From gamma = dh and Gamma = 2 deri as that call
 * returns them (device, K*K and K^4) and the context's integrals:
 *   fock[p][q] = F_pq = sum_r gamma_pr h_qr + sum_rst Gamma_prst (qr|st)
 *   grad[p][q] = dE/dkappa_pq = 2 (F_qp - F_pq)
 * the derivative of the energy at a fixed state when the orbitals are
 * rotated by U = exp(kappa), kappa antisymmetric (h -> U^T h U and likewise
 * for each index of (pq|rs)); device outputs, K*K each, fock may be NULL.
 * Synchronises the stream before returning. */
dmrg_status dmrg_orbital_gradient(dmrg_ctx ctx, const double* dh, const double* deri, double* fock,
                                  double* grad);

/* Truncates the optimised window psi (device, current window (i, i+1)) and
 * moves the window (two-site DMRG step; the truncation error of the Method
 * section).  The reduced density matrix of the half of the window left
 * behind is diagonalised per middle-bond sector and the max_bond_dim
 * largest eigenvalues over all sectors are kept (ties: lower sector, then
 * later index; eigenvalues below cutoff * largest are dropped).
 *   direction +1: site i becomes the new left-canonical tensor, the window
 *                 moves to (i+1, i+2); needs i+1 <= K-2.
 *   direction -1: site i+1 becomes the new right-canonical tensor, the
 *                 window moves to (i-1, i); needs i >= 1.
 * The guess for the new window (psi carried over, White's transformation) is
 * kept in the context: read it with dmrg_get_psi after dmrg_build_ops for the
 * new window.  trunc_err_out: discarded weight / total weight (may be NULL),
 * kept_out: new bond dimension (may be NULL).  Invalidates the cached block
 * operators that depend on the changed tensors. */
dmrg_status dmrg_truncate(dmrg_ctx ctx, const double* psi, int32_t direction, int32_t max_bond_dim,
                          double cutoff, double* trunc_err_out, int32_t* kept_out);

/* Copies the current window's guess left by dmrg_truncate (device pointer of
 * length dmrg_psi_size). */
dmrg_status dmrg_get_psi(dmrg_ctx ctx, double* out);

/* Checks a problem and (optionally, mps may be NULL) an MPS layout on the
 * host, without a context or a device: the ranges and parity of the active
 * space (N electrons in K orbitals, 2Sz), finite integrals, h symmetric and
 * (pq|rs) = (qp|rs) = (pq|sr) = (rs|pq) to 1e-10 of the largest entry (the
 * real-orbital Hamiltonian of the Method section), and for the MPS: K sites,
 * a window inside the chain, bond_offsets[0] = 0, every bond non-empty with
 * sorted unique sectors and positive dimensions, bond 0 = (0,0) and
 * bond K = (N, 2Sz) of dimension 1, and a non-NULL tensor with at least one
 * allowed block for every site outside the window.  dmrg_build_ops applies
 * the same checks.  Returns DMRG_ERR_INVALID_ARG or DMRG_ERR_SHAPE with the
 * message in dmrg_last_error(NULL). */
dmrg_status dmrg_validate(const dmrg_problem* problem, const dmrg_mps* mps);

/* The sectors of bond `bond` (0..K) of the context's current MPS, e.g. the
 * middle bond written by dmrg_truncate.  n_sectors receives the count; the
 * three arrays (host, capacity entries each) receive (N, 2Sz, dim) in
 * ascending order when non-NULL (all three or none). */
dmrg_status dmrg_get_bond(dmrg_ctx ctx, int32_t bond, int32_t capacity, int32_t* n_sectors,
                          int32_t* sector_n, int32_t* sector_2sz, int32_t* sector_dim);

/* The MPS site tensor `site` of the context (the updated site out of a
 * two-site step: after dmrg_truncate with direction +1 the new left-canonical
 * tensor of the old window's left site, with -1 the new right-canonical tensor
 * of its right site; the A of eq. (1) in the layout of dmrg_mps.site_data:
 * blocks (l, n) -> r ascending by l then n, each d_l x d_r row-major, with
 * the bonds of dmrg_get_bond).  size receives the number of doubles; out
 * (host, capacity doubles) receives the tensor when non-NULL.  The window's
 * two sites are held in psi and are refused (DMRG_ERR_STATE).  Synchronises
 * the context stream. */
dmrg_status dmrg_get_site(dmrg_ctx ctx, int32_t site, int64_t capacity, double* out, int64_t* size);

/* Energy functional of a window vector (Method section: the energy of the
 * MPS of eq. (1) with psi at the current window):
 *   energy = psi^T H_eff psi + e_core psi^T psi,   norm2 = psi^T psi
 * with sigma = H_eff psi in the given precision and both dot products in
 * FP64 on the device (for normalised psi, the energy).  psi, sigma_out and
 * grad_psi are device pointers of dmrg_psi_size doubles; sigma_out (may be
 * NULL) receives sigma, grad_psi (may be NULL) the gradient
 * d energy / d psi = 2 (sigma + e_core psi).  h and eri (host, K*K and K^4,
 * both or neither) are compared with the integrals the operators were built
 * from: a difference above 1e-13 of the largest entry is DMRG_ERR_INVALID_ARG,
 * so a caller cannot take the energy of one Hamiltonian with the operators of
 * another.  energy_out and norm2_out (may be NULL) are host pointers;
 * synchronises the context stream. */
dmrg_status dmrg_energy(dmrg_ctx ctx, const double* h, const double* eri, const double* psi,
                        int32_t precision, double* sigma_out, double* grad_psi, double* energy_out,
                        double* norm2_out);

/* ---- spin adaptation (SU(2)): the contraction of a spin-adapted sigma ----
 *
 * Spin-adapted DMRG counts bond states in multiplets (Numerical procedure
 * section: fixed D_SU(2), Fig. 2-3).  The window vector of total N and spin
 * S is stored reduced, over coupled blocks (a, b) of a left multiplet sector
 * a = (N_a, 2S_a, d_a) and a right sector b with N_a + N_b = N and S in
 * S_a x S_b: the blocks in order of a, then b, each d_a x d_b row-major
 * (dmrg_su2_psi_size gives the length).  A spin-adapted sigma is a sum of
 * scalar products c [A^k x B^k]^0 of a left and a right tensor operator of
 * rank k (k = 0, 1/2, 1, ...), given by their reduced matrices in the
 * Clebsch-Gordan convention of the Wigner-Eckart theorem,
 * <a' S' M'|T^k_q|a S M> = <S M; k q|S' M'> <a' S'||T^k||a S>.  Block by
 * block,
 *   sigma[a', b'] += c (-1)^(p N_a) W A[a', a] psi[a, b] B[b', b]^T,
 *   W = (-1)^(S_a + S_b' + S + k) sqrt((2S_a'+1)(2S_b'+1)/(2k+1))
 *       {S_a S_b S; S_b' S_a' k}   (a Wigner 6j symbol),
 * p the fermion parity of B and N_a the electrons of the ket's left part.
 * The library runs it as two stages of its FP64 grouped GEMM (T = psi B^T,
 * then sigma += W c A T).  Building the spin-adapted operators of a
 * Hamiltonian (renormalisation with 9j recoupling) is not part of the
 * library: the operators are the caller's. */
typedef struct {
  int32_t n_left, n_right;      /* multiplet sectors of the left / right block */
  const int32_t* left_n;        /* host arrays of n_left entries: N, 2S, dimension */
  const int32_t* left_two_s;
  const int32_t* left_dim;
  const int32_t* right_n;       /* host arrays of n_right entries */
  const int32_t* right_two_s;
  const int32_t* right_dim;
  int32_t n_elec, two_s;        /* total N and 2S of the window */
} dmrg_su2_window;

typedef struct {
  int32_t n_blocks;
  const int32_t* out_sector;    /* host: sector of the block's rows (bra) */
  const int32_t* in_sector;     /* host: sector of its columns (ket) */
  const int64_t* offset;        /* host: element offset of the block in data */
  const double* data;           /* device: blocks d_out x d_in row-major */
} dmrg_su2_operator;

typedef struct {
  int32_t left_op, right_op;    /* indices into the operator arrays */
  int32_t two_k;                /* rank k, doubled */
  int32_t parity;               /* fermion parity of the right operator (0, 1) */
  double coef;
} dmrg_su2_pair;

/* Length of the reduced window vector; host only, no context.  Errors:
 * DMRG_ERR_INVALID_ARG for a NULL pointer, a non-positive dimension, a
 * sector whose 2S and N differ in parity or a negative N or 2S. */
dmrg_status dmrg_su2_psi_size(const dmrg_su2_window* window, int64_t* n);

/* sigma = sum over pairs of c [A^k x B^k]^0 psi (the rule above) in FP64.
 * psi, sigma: device pointers of dmrg_su2_psi_size elements, caller-owned;
 * operators: host descriptors of device blocks (a block whose sectors or
 * ranks cannot couple contributes nothing).  Errors: DMRG_ERR_INVALID_ARG for
 * an invalid window, an operator index out of range, a block sector out of
 * range, or a pair whose right parity is not 0 or 1.  One call is
 * dmrg_su2_plan_create, dmrg_su2_plan_sigma and dmrg_su2_plan_destroy; it
 * synchronises the context stream before returning. */
dmrg_status dmrg_su2_sigma(dmrg_ctx ctx, const dmrg_su2_window* window, int32_t n_left_ops,
                           const dmrg_su2_operator* left_ops, int32_t n_right_ops,
                           const dmrg_su2_operator* right_ops, int32_t n_pairs,
                           const dmrg_su2_pair* pairs, const double* psi, double* sigma);

/* A spin-adapted sigma planned once and applied many times (the Davidson
 * iterations of one window).  dmrg_su2_plan_create checks its arguments as
 * dmrg_su2_sigma does, selects the block products that some pair needs,
 * splits the right operators into chunks whose stage-1 products fit the
 * context's workspace budget (8 GiB, DMRG_WS_BUDGET_MB at dmrg_create), and
 * uploads the GEMM descriptors.  The plan keeps the device addresses of the
 * operator blocks: their memory must stay allocated and unchanged while the
 * plan lives.  It owns device copies of psi and sigma and the workspace.
 * A plan belongs to its context: it is used and destroyed through that
 * context, and dmrg_destroy releases plans still alive (their handles then
 * become invalid).  precision: DMRG_FP64, or DMRG_BF16X3 (split-BF16
 * products with FP32 accumulation, flushed into FP64 per segment: the
 * plan packs the operator blocks once into BF16 hi/lo copies, rows padded
 * to 8 elements, and psi on every call; the Mixed precision section).
 * Errors: those of dmrg_su2_sigma; DMRG_ERR_INVALID_ARG for another
 * precision; DMRG_ERR_OOM when device memory runs out. */
typedef struct dmrg_su2_plan_s* dmrg_su2_plan;
dmrg_status dmrg_su2_plan_create(dmrg_ctx ctx, const dmrg_su2_window* window, int32_t n_left_ops,
                                 const dmrg_su2_operator* left_ops, int32_t n_right_ops,
                                 const dmrg_su2_operator* right_ops, int32_t n_pairs,
                                 const dmrg_su2_pair* pairs, int32_t precision, dmrg_su2_plan* plan);

/* sigma = the plan's contraction of psi (device pointers of psi_size
 * elements, caller-owned; sigma may be psi itself).  Stream-ordered on the
 * context stream, no synchronisation, no allocation.  Calls on one plan run
 * in stream order; psi and sigma may be reused once the stream reaches the
 * end of the call.  DMRG_ERR_INVALID_ARG for a plan that is not one of
 * this context's. */
dmrg_status dmrg_su2_plan_sigma(dmrg_ctx ctx, dmrg_su2_plan plan, const double* psi, double* sigma);

typedef struct {
  int64_t psi_size;        /* elements of psi and sigma */
  int32_t n_chunks;        /* workspace chunks (stage-1 + stage-2 launch pairs) */
  int32_t pad;
  int64_t n_segments;      /* block products of both stages */
  int64_t workspace_bytes; /* stage-1 workspace (the largest chunk; BF16 hi + lo for DMRG_BF16X3) */
  double flops_stage1;     /* 2 d_a d_b d_b' per stage-1 product */
  double flops_stage2;     /* 2 d_a' d_a d_b' per stage-2 product */
} dmrg_su2_info;
dmrg_status dmrg_su2_plan_info(dmrg_ctx ctx, dmrg_su2_plan plan, dmrg_su2_info* out);

/* Synchronises the context stream, then releases the plan.  A NULL plan is
 * a no-op. */
dmrg_status dmrg_su2_plan_destroy(dmrg_ctx ctx, dmrg_su2_plan plan);

/* The renormalisation step of spin-adapted operators (Numerical procedure
 * section): the reduced blocks of the coupled product X^k = [A^k1 x B^k2]^k
 * of an operator A on subsystem 1 (a block) and B on subsystem 2 (a site,
 * or any second block),
 *   <(a' S_a', b' S_b') S' || X^k || (a S_a, b S_b) S>
 *     = (-1)^(p(B) N_a) sqrt((2S + 1)(2k + 1)(2S_a' + 1)(2S_b' + 1))
 *       {S_a' S_a k1; S_b' S_b k2; S' S k} <a'||A||a> <b'||B||b>
 * (a Wigner 9j symbol; reduced elements in the Clebsch-Gordan convention of
 * dmrg_su2_sigma).  The coupled sectors of the two subsystems are (i1, i2,
 * 2S) for every sector i1 of subsystem 1, i2 of subsystem 2 and S in
 * S_i1 x S_i2, numbered in that order (i1 slowest, then i2, then 2S
 * ascending); a coupled sector holds d_i1 d_i2 multiplets, (alpha1, alpha2)
 * with alpha1 slowest.  sectors: the left arrays of the window describe
 * subsystem 1, the right arrays subsystem 2 (n_elec and two_s are not
 * used).  An output block is the Kronecker product of one block of A and
 * one of B, scaled; blocks are ordered by A's block, then B's, then 2S,
 * then 2S'; blocks whose coefficient vanishes are left out.
 * dmrg_su2_product_size (host only; a and b need only their sector arrays)
 * gives the number of output blocks and of output elements;
 * dmrg_su2_product writes the blocks' sectors and element offsets (host
 * arrays of n_blocks) and their data (device, n_elems, row-major blocks),
 * synchronising the context stream.  Errors: DMRG_ERR_INVALID_ARG for an
 * invalid sector list, a block sector out of range, negative ranks or a
 * parity other than 0 or 1. */
dmrg_status dmrg_su2_product_size(const dmrg_su2_window* sectors, const dmrg_su2_operator* a,
                                  const dmrg_su2_operator* b, int32_t two_k1, int32_t two_k2,
                                  int32_t two_k, int32_t* n_blocks, int64_t* n_elems);
dmrg_status dmrg_su2_product(dmrg_ctx ctx, const dmrg_su2_window* sectors, const dmrg_su2_operator* a,
                             const dmrg_su2_operator* b, int32_t two_k1, int32_t two_k2, int32_t two_k,
                             int32_t parity_b, int32_t* out_sector, int32_t* in_sector, int64_t* offset,
                             double* data);

/* The renormalisation's projection onto the kept multiplets: the coupled
 * sectors c of the enlarged block (as numbered by dmrg_su2_product) are
 * grouped into new sectors g of one (N, S) each; the kept multiplets of g
 * are the columns of U_g (rows: the multiplets of g's coupled sectors in
 * their order), and proj[c] is the block of U_g's rows that belong to c
 * (d_c x D_g, row-major, device).  For operator blocks X[c', c] the result
 * is O[g', g] = sum over the blocks with c' in g' and c in g of
 * proj[c']^T X[c', c] proj[c] (D_g' x D_g), by two stages of the FP64
 * grouped GEMM.  Output blocks are ordered by g', then g. */
typedef struct {
  int32_t n_coupled;
  const int32_t* coupled_dim;   /* host, n_coupled: multiplets of each coupled sector */
  const int32_t* coupled_group; /* host, n_coupled: its new sector, or -1 if kept out */
  int32_t n_groups;
  const int32_t* group_dim;     /* host, n_groups: kept multiplets D_g */
  const double* const* proj;    /* host array of n_coupled device pointers (NULL where kept out) */
} dmrg_su2_basis;

/* Number of output blocks and elements (host only; proj is not read).
 * Errors: DMRG_ERR_INVALID_ARG for a sector or group index out of range or
 * a non-positive dimension. */
dmrg_status dmrg_su2_rotate_size(const dmrg_su2_basis* basis, int32_t n_blocks, const int32_t* out_sector,
                                 const int32_t* in_sector, int32_t* n_out, int64_t* n_elems);

/* Writes the output blocks' groups and element offsets (host arrays of
 * n_out) and data (device, n_elems); X is given as dmrg_su2_product
 * returns it (host sector and offset arrays, device data).  Synchronises
 * the context stream (its workspace is released on return). */
dmrg_status dmrg_su2_rotate(dmrg_ctx ctx, const dmrg_su2_basis* basis, int32_t n_blocks, const int32_t* out_sector,
                            const int32_t* in_sector, const int64_t* offset, const double* data,
                            int32_t* out_group, int32_t* in_group, int64_t* out_offset, double* out_data);

/* Diagnostic: copies diag(H_eff) of the current window (the Davidson
 * preconditioner; psi layout, device pointer, length dmrg_psi_size). */
dmrg_status dmrg_debug_diag(dmrg_ctx ctx, double* out);

/* Diagnostic: C = alpha * op(A) op(B) + beta * C with the library's grouped
 * GEMM kernel of the given precision, for kernel-level numerics tests.
 * A is m x k (stored k x m when trans_a), B is k x n (stored n x k when
 * trans_b); row-major device pointers with leading dimensions lda, ldb, ldc.
 * beta must be 0 or 1.  Stream-ordered, no synchronisation. */
dmrg_status dmrg_debug_gemm(dmrg_ctx ctx, int32_t m, int32_t n, int32_t k, const double* a,
                            int32_t lda, int32_t trans_a, const double* b, int32_t ldb,
                            int32_t trans_b, double* c, int32_t ldc, double alpha, int32_t beta,
                            int32_t precision);

#ifdef __cplusplus
}
#endif

#endif /* DMRG_H */
