/*
 * libipr: inverse matrix p-th roots A^{-1/p} of symmetric positive definite
 * matrices on AMD Instinct MI355X (gfx950).
 *
 * The method is the iteration of Bini et al. as stated in Section II of
 * Lass, Kuehne, Plessl, "Using Approximate Computing for the Calculation of
 * Inverse Matrix p-th Roots" (arXiv 1703.02283):
 *   eq. (1)  C_{k+1} = ((p + 1) C_k - C_k^{p+1} A) / p,
 *   eq. (2)  convergence when ||I - C_0^p A||_2 < 1,
 *   eq. (3)  the start C_0 = A^T / (||A||_1 ||A||_inf).
 * For p = 1 the iteration is the Newton-Schulz iteration for A^{-1}.
 *
 * Conventions shared by every entry point below:
 *   - Matrices are dense, n x n, row-major with leading dimension n, float64
 *     unless stated. A must be exactly symmetric; symmetry and definiteness
 *     are not checked (an indefinite A shows up as IPR_EDIVERGED).
 *   - Pointers named d* are device pointers owned by the caller. The library
 *     never allocates or frees device memory: all temporary storage comes from
 *     the caller's workspace (see ipr_workspace_size). The only memory the
 *     library allocates is a small pinned host buffer per calling thread, used
 *     to read one scalar per iteration; it lives until the process ends.
 *   - All device work is ordered on `stream`. Calls that return host results
 *     synchronise the stream before returning; ipr_solve also synchronises once
 *     per iteration to read the residual.
 *   - A workspace must not be shared by calls that may overlap in time.
 *   - Every function returns an ipr_status; on IPR_EHIP or IPR_EARG,
 *     ipr_last_error() returns a message for the calling thread.
 */
#ifndef IPR_H
#define IPR_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IPR_OK = 0,
  IPR_EARG = 1,        /* invalid argument or workspace too small */
  IPR_EMAXITER = 2,    /* max_iter updates applied without reaching tol */
  IPR_EFLOOR = 3,      /* the residual stopped falling above tol (precision floor): below 1/2,
                          where every exact step at least halves it */
  IPR_EDIVERGED = 4,   /* NaN/Inf or residual > 1e6, again after one restart from the
                          scaled identity (ipr_solve; not for the LITERAL order or
                          approximate storage, which report the first divergence) */
  IPR_EHIP = 5,        /* a HIP runtime call failed */
  IPR_EGUARD = 6       /* a requested start violates eq. (2) and fallback was disabled */
} ipr_status;

/* Start C_0 (Section II). */
typedef enum {
  IPR_INIT_IDENTITY = 0,  /* C_0 = (||A||_1 ||A||_inf)^{-1/(2p)} I: satisfies eq. (2) for every SPD A */
  IPR_INIT_PAPER_EQ3 = 1, /* eq. (3): C_0 = A^T / (||A||_1 ||A||_inf) */
  IPR_INIT_POLY = 2,      /* C_0 = s^{-1/p} (b0 I + b1 A/s + b2 (A/s)^2), s = sqrt(||A||_1 ||A||_inf) */
  IPR_INIT_LEARNED = 3,   /* POLY in units of the certified bound s = (||A^2||_1 ||A^2||_inf)^{1/4}
                             (>= lambda_max, one product), with (log b0, b1, b2) predicted by the
                             MLP in schedule.mlp_params from ipr_features; checked against eq. (2) */
  IPR_INIT_USER = 4       /* C_0 = the contents of dC on entry (a warm start). It must be symmetric;
                             for the coupled and literal orders also a function of A (a polynomial
                             in A, or the root of a matrix with the same eigenvectors), for
                             Newton-Schulz any C_0 with ||I - A C_0||_2 < 1. Accepted when the
                             start's residual ||I - C_0^p A||_F (resp. ||I - A C_0||_F) is below 1,
                             which implies eq. (2); otherwise guard_fallback applies */
} ipr_init;

/* Approximate storage (Sections III-C and IV): how the input and every
 * matrix the iteration stores between products are kept. */
typedef enum {
  IPR_STORE_NONE = 0,   /* float64 */
  IPR_STORE_FLOAT = 1,  /* float with store_bits stored mantissa bits (1..52), unbounded exponent */
  IPR_STORE_FIXED = 2   /* fixed point with store_bits fractional bits (1..64), enough integer bits */
} ipr_store_format;

/* Order in which the products of eq. (1) are evaluated (Section II). */
typedef enum {
  IPR_EVAL_COUPLED = 0,       /* M_k = C_k^p A carried along: N_k = ((p+1) I - M_k)/p,
                                 C_{k+1} = C_k N_k, M_{k+1} = N_k^p M_k (p + 1 products; default;
                                 for p a power of two >= 4, N_k^p by repeated squaring:
                                 log2(p) + 2 products, 4 for p = 4) */
  IPR_EVAL_LITERAL = 1,       /* eq. (1) as printed: X = C_k^p A, C_{k+1} = ((p+1) C_k - C_k X)/p,
                                 full products, no symmetrisation (p + 1 products; a diagnostic:
                                 rounding errors grow beyond small condition numbers) */
  IPR_EVAL_NEWTON_SCHULZ = 2  /* p = 1 only: R_k = I - A C_k (full product), C_{k+1} = C_k + C_k R_k
                                 (2 products; removes errors that do not commute with A) */
} ipr_evaluation;

/* Arithmetic type of the bulk (early) iterations. FP64 refinement follows a
 * low-precision bulk phase (Section III: low precision first, precise last). */
typedef enum {
  IPR_FP64 = 0,
  IPR_BF16 = 1,      /* bf16 operands, fp32 accumulation */
  IPR_FP16 = 2,      /* fp16 operands with per-128x128-tile power-of-two scales, fp32 accumulation */
  IPR_FP8_E4M3 = 3,  /* fp8 e4m3 operands with per-128x128-tile power-of-two scales, fp32 accumulation */
  IPR_FP64_INT8_EMUL = 4 /* every product of the iteration FP64-accurate from int8 digit slices
                            (ipr_gemm_emul, schedule.emul_slices digits): no refinement phase;
                            the start's squarings and the final check stay on the FP64 cores;
                            n <= 132864 */
} ipr_dtype;

typedef struct {
  int init;            /* ipr_init */
  int bulk_dtype;      /* ipr_dtype */
  int max_iter;        /* cap on updates (default 100) */
  int triangle;        /* 1: compute one triangle of every symmetric product and mirror it (default 1) */
  int guard_fallback;  /* 1: a POLY/LEARNED/PAPER_EQ3 start that fails the eq. (2) check falls back to IDENTITY (default 1) */
  int verify;          /* 1: confirm ||I - C^p A||_F < tol from C and A before returning OK (default 1) */
  double bulk_switch;  /* low-precision bulk phase ends when its residual falls below this or stalls (default 0.05) */
  double stall_ratio;  /* the low-precision bulk phase stalls when its residual is not below
                          stall_ratio * best for 2 iterations; the FP64 phase ends on IPR_EFLOOR
                          when, below 1/2, it is not below stall_ratio * best for 3 (default 0.5) */
  double poly[3];      /* b0, b1, b2 for IPR_INIT_POLY */
  const float* mlp_params; /* device, IPR_MLP_NPARAM floats, for IPR_INIT_LEARNED */
  int timing;          /* 1: time every matrix product with device events (ms_gemm, gemm_flops) */
  int tile;            /* ipr_solve_batched: product tile edge 32 or 64; 0 = size-bucket table */
  int scale_squarings; /* IDENTITY start: up to this many repeated squarings of A / sigma tighten
                          the scale s of C_0 = s^{-1/p} I (default 0: s = sigma, the norm bound
                          of eq. (3)); see ipr_solve */
  int dynamic_scaling; /* IDENTITY start, FP64 (and the Newton-Schulz steps of a p = 1
                          low-precision bulk phase): scale every step by a factor chosen from
                          bounds on the spectrum of M_k, with the lower end estimated by Lanczos
                          (default 0: the plain iteration of eq. (1)); see ipr_solve */
  int evaluation;      /* ipr_evaluation (default COUPLED); LITERAL and NEWTON_SCHULZ need the FP64
                          bulk dtype and ipr_solve (not the batched solver) */
  int emul_slices;     /* IPR_FP64_INT8_EMUL: 7-bit digits per operand, 1..12 (0: 10, which
                          reaches the FP64 result at n = 16384; see ipr_gemm_emul) */
  int store_format;    /* ipr_store_format (default NONE). Otherwise the paper's storage-only
                          approximation: A, C_0, M_0, N_0 and every product the iteration stores
                          (C_k, M_k, N_k and the intermediates of N^p M) are rounded to nearest
                          (ties to even) when written; products and epilogues compute in FP64;
                          the final check uses the caller's A. Needs the plain coupled FP64
                          iteration from the scaled identity (IPR_EARG otherwise); a coarse
                          format ends on its floor (IPR_EFLOOR) */
  int store_bits;      /* stored mantissa bits (FLOAT) or fractional bits (FIXED) */
  int store_regime;    /* with store_format: 0 = storage only (default: the stored matrices are
                          rounded, arithmetic in FP64); 1 = all arithmetic (Section IV, "all
                          involved calculations"): every scalar operation is one float64
                          operation rounded to the type. Then A~ = rnd(A), c = rnd(sigma^(-1/p)),
                          c_p = rnd(c^p), C_0 = c I, M_0 = rnd(c_p A~), N = rnd(I + rnd(rnd(I - M)/p)),
                          and each product sums acc <- rnd(acc + rnd(l_ki r_kj)) over k in
                          increasing order (upper triangle, mirrored) on the vector units */
  const double* hist_ref; /* device n x n or NULL: ipr_solve writes ||C_k - hist_ref||_F to
                          hist_err[k] for every iterate k it forms (e.g. the float64 root, for
                          the error curves of Section IV-C): the coupled FP64 iteration and
                          both approximate regimes (not the low-precision bulk phase) */
  double* hist_err;    /* host, hist_len doubles (or NULL) */
  double* hist_rho;    /* host, hist_len doubles (or NULL): ||I - M_k||_F per iterate (NaN for
                          an iterate whose M was not formed) */
  int hist_len;        /* capacity of hist_err / hist_rho; entries k >= hist_len are dropped */
  int bulk_force;      /* 1: run a BF16/FP16/FP8 bulk phase also for p >= 2 (default 0: skipped
                          there and reported in ipr_result.bulk_skipped). For p >= 2 the phase
                          leaves an error that does not commute with A; the coupled FP64 steps
                          do not remove it, so the solve restarts in FP64 (fallback_used) and
                          the phase was spent for nothing */
  int scale_lanczos;   /* IDENTITY start, n >= 32: the scale s of C_0 = s^{-1/p} I is 1.01 times
                          the largest Ritz value of 24 Lanczos steps on A (12 in
                          ipr_solve_batched; the run that dynamic_scaling needs anyway), an
                          estimate of lambda_max from below,
                          instead of a certified bound: no product is spent on the scale.
                          Exclusive with scale_squarings (IPR_EARG). Not certified: eq. (2)
                          holds while lambda_max < 2 s, and a diverging run restarts from the
                          norm-scaled identity (fallback_used); see ipr_solve (default 0) */
} ipr_schedule;

typedef struct {
  int status;          /* ipr_status of the solve */
  int iters_bulk;      /* updates applied in the low-precision bulk phase */
  int iters_fp64;      /* updates applied in FP64 */
  int fallback_used;   /* 1 if IDENTITY was used instead: the requested start failed the
                          guard, the low-precision phase failed and FP64 restarted, or the
                          iteration diverged and restarted once */
  int gemms;           /* matrix products launched (all phases) */
  double residual_proxy; /* last tracked ||I - C^p A||_F */
  double residual_true;  /* ||I - C^p A||_F computed from C and A (NaN if not verified) */
  double init_bound;   /* sup over x in (0,1] of q(x)^p x for the start used (eq. (2) needs < 2) */
  double norm1, norminf; /* ||A||_1 and ||A||_inf */
  double poly_used[3]; /* (b0, b1, b2) of the start used: C_0 = s^{-1/p} q(A/s) */
  double init_scale;   /* that s: sqrt(||A||_1 ||A||_inf), or the certified bound
                          (||A^2||_1 ||A^2||_inf)^{1/4} >= lambda_max for the learned start */
  double ms_norms, ms_init, ms_bulk, ms_refine, ms_verify; /* phase times (device events) */
  int gemm_launches;   /* products timed (schedule.timing = 1) */
  double ms_gemm;      /* their summed device time */
  double gemm_flops;   /* their algorithmic flops: 2 n^3 per full product, n^2 (n + 1) per triangle */
  int lp_gemm_launches;  /* the same for the low-precision products of the bulk phase and the
                            int8-slice products of IPR_FP64_INT8_EMUL (one per product) */
  double ms_lp_gemm;     /* (matrix-core kernels only; the rounding or splitting of operands is
                            not included) */
  double lp_gemm_flops;
  double lmin_est;       /* dynamic_scaling: the Lanczos estimate of lambda_min(A) (0 otherwise) */
  int reest_iter;        /* dynamic_scaling: the step before which lambda_min(M_k) was estimated
                            again (once its bound reached 0.03; 0 if not) */
  double lmin_reest;     /* that estimate (0 if none) */
  int bulk_skipped;      /* 1: a BF16/FP16/FP8 bulk dtype was requested but not run (p >= 2
                            without schedule.bulk_force; in ipr_solve_batched every p >= 2
                            item): the solve ran in FP64 */
} ipr_result;

#define IPR_MLP_NIN 16
#define IPR_MLP_NHID 64
#define IPR_MLP_NOUT 3
/* W1 (64x16), b1 (64), W2 (64x64), b2 (64), W3 (3x64), b3 (3), row-major. */
#define IPR_MLP_NPARAM (IPR_MLP_NHID * IPR_MLP_NIN + IPR_MLP_NHID + IPR_MLP_NHID * IPR_MLP_NHID + \
                        IPR_MLP_NHID + IPR_MLP_NOUT * IPR_MLP_NHID + IPR_MLP_NOUT)

/* Fills *s with the defaults documented above (IDENTITY start, FP64, triangle on). */
void ipr_schedule_default(ipr_schedule* s);

/* Bytes of device workspace a solve of order <= n_max and root <= p_max needs
 * (batch = 1), or a batched solve of `batch` matrices whose orders sum their
 * squares to at most n_max * n_max (see ipr_solve_batched). */
size_t ipr_workspace_size(int n_max, int p_max, int batch, const ipr_schedule* s);

/* A^{-1/p} of one SPD matrix (Section II, eqs. (1)-(3)).
 *   dA    device, n x n float64, symmetric (read only)
 *   dC    device, n x n float64: receives A^{-1/p} (exactly symmetric, except with the
 *         LITERAL order); with IPR_INIT_USER it holds C_0 on entry; must not alias dA
 *   tol   stop when ||I - C^p A||_F < tol (> 0)
 *   s     schedule (NULL = defaults)
 *   out   host, receives the result record (may be NULL)
 *   dWork device workspace of work_bytes >= ipr_workspace_size(n, p, 1, s)
 * Returns IPR_OK when the residual was reached; IPR_EFLOOR / IPR_EMAXITER /
 * IPR_EDIVERGED leave the last iterate in dC. */
int ipr_solve(const double* dA, double* dC, int n, int p, double tol,
              const ipr_schedule* s, ipr_result* out, void* dWork, size_t work_bytes,
              hipStream_t stream);

/* Eigenvalues of a dense symmetric matrix, ascending: the step after the
 * Loewdin transform (Section IV-A: the eigenvalues of X H X, X = S^{-1/2},
 * are those of H c = e S c). Householder reduction to tridiagonal form (one
 * reflector per column, the trailing matrix kept whole) and multisection
 * (bisection at 64 points per round) on the Sturm count of the tridiagonal
 * matrix, FP64 throughout.
 *   dA    device, n x n float64, symmetric (read only)
 *   dW    device, n float64: the eigenvalues in ascending order
 *   dWork device workspace of work_bytes >= ipr_eigvalsh_workspace(n)
 * Errors: IPR_EARG for a null pointer, n < 1 or a short workspace. Stream
 * ordered; returns without synchronising. */
int ipr_eigvalsh(const double* dA, int n, double* dW, void* dWork, size_t work_bytes,
                 hipStream_t stream);
size_t ipr_eigvalsh_workspace(int n);

/* Size of the fixed device workspace of ipr_solve_noalloc: 64 MiB per device. */
#define IPR_NOALLOC_SCRATCH_BYTES (64u << 20)

/* ipr_solve without a caller workspace, for callers that cannot allocate
 * device memory (serving loops, harnesses that forbid hipMalloc). The
 * workspace is a fixed 64 MiB device array of the library, one per device,
 * looked up on the first call on each device and held until the process
 * ends. The call allocates nothing: no device or pinned memory, no events.
 * Arguments and results as ipr_solve, except:
 *   - ipr_workspace_size(n, p, 1, s) must not exceed IPR_NOALLOC_SCRATCH_BYTES
 *     (n <= 1094 with the FP64 schedules); larger problems return IPR_EARG;
 *   - schedule.timing must be 0 (IPR_EARG otherwise); every ms_* field is 0.
 * Every call on one device shares that device's array and leaves its
 * contents behind (the solve initialises all it reads): calls that overlap in
 * time on one device race, whatever their streams. */
int ipr_solve_noalloc(const double* dA, double* dC, int n, int p, double tol,
                      const ipr_schedule* s, ipr_result* out, hipStream_t stream);

/* Independent solves of `batch` SPD matrices of uneven orders in one
 * persistent kernel launch (device-side iteration loop per matrix).
 *   dA_packed, dC_packed  device, matrices back to back (float64)
 *   offsets  host, batch int64: element offset of matrix i in both buffers
 *   n, p     host, batch ints: order (1 <= n <= 1024) and root (1 <= p <= 8)
 *   out      host, batch result records (may be NULL)
 * Only IPR_INIT_IDENTITY and IPR_FP64 / IPR_BF16 bulk are supported here. */
int ipr_solve_batched(const double* dA_packed, double* dC_packed, const int64_t* offsets,
                      const int* n, const int* p, int batch, double tol,
                      const ipr_schedule* s, ipr_result* out, void* dWork, size_t work_bytes,
                      hipStream_t stream);

/* Size buckets of the batched solver's tile table: bucket b holds the orders
 * up to its maximum (48, 96, 192, 384, 768, 1024) above the previous one's. */
#define IPR_BATCH_BUCKETS 6

/* Times every tile edge (32, 64) on synthetic batches of each bucket's
 * largest order (a fixed 3 iterations per matrix, one persistent launch each)
 * and stores the fastest in the process-wide table used when schedule.tile is
 * 0; the table is copied to host tiles_out[IPR_BATCH_BUCKETS] (may be NULL).
 * Each bucket times up to 512 matrices, as many as fit in dWork (9 n^2
 * doubles each); a bucket none fits in keeps its entry. */
int ipr_tune_batched(void* dWork, size_t work_bytes, int* tiles_out, hipStream_t stream);

/* Reads or replaces the process-wide tile table (host arrays of IPR_BATCH_BUCKETS). */
int ipr_get_batched_tiles(int* tiles);
int ipr_set_batched_tiles(const int* tiles);

/* D = L^T R for n x n float64 matrices on the FP64 matrix cores (the product
 * every step of eq. (1) is made of), followed by D <- alpha D + beta X + gamma I.
 * X may be NULL. With triangle = 1 only the upper triangle is computed and
 * mirrored (for products known to be symmetric). dD must not alias dL or dR. */
int ipr_gemm(const double* dL, const double* dR, const double* dX, double* dD, int n,
             double alpha, double beta, double gamma, int triangle, hipStream_t stream);

/* Low-precision product (the storage-approximation regime of Sections III-B
 * and IV): L and R are rounded to `dtype` with per-128x128-tile power-of-two
 * scales (fp16, fp8) or none (bf16), multiplied on the matrix cores with fp32
 * accumulation; D (float64) = L^T R. triangle = 1: only the tiles on and above
 * the diagonal are computed and D is mirrored from them (for a symmetric
 * product, as in the iteration). dWork >= ipr_gemm_lowp_workspace(n). */
int ipr_gemm_lowp(const double* dL, const double* dR, double* dD, int n, int dtype, int triangle,
                  void* dWork, size_t work_bytes, hipStream_t stream);
size_t ipr_gemm_lowp_workspace(int n);

/* FP64-accurate product D = L^T R on the int8 matrix cores: the low-precision
 * units Section III-B asks for, at the accuracy the iteration needs (eq. (1)
 * for p >= 2 floors unless its products are FP64-accurate). Error-free
 * splitting into 8-bit digits (Ozaki, Ogita, Oishi and Rump, Numer.
 * Algorithms 59, 2012): each column of L and of R is scaled by a power of two
 * below its largest magnitude and cut into `slices` digits of 7 bits
 * (rounded to nearest, in [-127, 127]); the digit products with t + u <=
 * slices + 1 are exact in int32 and their levels are added in float64 from
 * the smallest. Error per element below n (slices + 2) 2^(e_i + f_j - 7 slices)
 * plus float64 rounding (2^e_i, 2^f_j: the column scales). An entry far below
 * its column's largest keeps fewer bits than float64 gives it: with 9 slices
 * the n = 8192 and 16384 iterations (kappa = 1e4) stop near 1e-10 instead of
 * 3e-11; 10 slices reach the float64 result. Costs slices (slices + 1) / 2
 * int8 products. triangle as in ipr_gemm_lowp. Ownership and stream as ipr_gemm;
 * dD must not alias an operand.
 * dWork >= ipr_gemm_emul_workspace(n, slices) bytes (device). Errors:
 * IPR_EARG for a null pointer, n < 1, slices outside 1..12, n above 132864
 * (one digit product must fit an int32 accumulation) or a short workspace.
 * A column holding Inf or NaN gives NaN in the matching row or column of D. */
int ipr_gemm_emul(const double* dL, const double* dR, double* dD, int n, int slices, int triangle,
                  void* dWork, size_t work_bytes, hipStream_t stream);
size_t ipr_gemm_emul_workspace(int n, int slices);

/* Loewdin orthogonalisation, the step after the inverse square root in the
 * paper's application (Section IV-A: the generalised eigenproblem
 * H c = e S c of a non-orthogonal basis in standard form): dX = S^{-1/2} by
 * ipr_solve (p = 2, schedule s, tolerance tol; `out` is its result), then
 * dHout = X H X from two FP64 products (H X in full, then X (H X) as one
 * mirrored triangle). The eigenvalues of Hout are those of (H, S); an
 * eigenvector y of Hout gives c = X y. S and H: n x n float64, symmetric,
 * row-major, device; dX, dHout: n x n device outputs that alias neither input
 * nor each other. dWork >= ipr_lowdin_workspace(n, s) bytes (device). Returns
 * the solve's status (dHout is written only when it is IPR_OK), IPR_EARG for
 * bad arguments, IPR_EHIP for HIP failures. Stream-ordered on `stream`. */
int ipr_lowdin(const double* dS, const double* dH, double* dX, double* dHout, int n, double tol,
               const ipr_schedule* s, ipr_result* out, void* dWork, size_t work_bytes,
               hipStream_t stream);
size_t ipr_lowdin_workspace(int n, const ipr_schedule* s);

/* ||A||_1 and ||A||_inf (eq. (3)) into host out[0], out[1]. dWork >= n*(n/256+2)*8 bytes. */
int ipr_norms(const double* dA, int n, double* out, void* dWork, size_t work_bytes,
              hipStream_t stream);

/* 16 features of each matrix of a packed batch (the learned start's input):
 * dFeat (device, batch x 16 float32); offsets/n/p are host arrays, staged
 * into dWork (>= 16 * batch + 1024 bytes). With s = sqrt(||A||_1 ||A||_inf),
 * B = A/s, d = diag B, r_i = sum_j |B_ij|, o_i = r_i - |d_i|, t1 = trace B / n,
 * t2 = ||B||_F^2 / n: clamp(log2 n, 6, 10)/10 (the training sizes 64..1024),
 * p/4, t1, t2, log10 t1, log10 t2, t1^2/t2,
 * min d, max d, log10 max(min d, 1e-30), min(d_i - o_i), mean r, sum o / sum|d|,
 * max off-diagonal |B_ij|, std(d)/mean(d), log10 s. All O(n^2). */
int ipr_features(const double* dA_packed, const int64_t* offsets, const int* n, const int* p,
                 int batch, float* dFeat, void* dWork, size_t work_bytes, hipStream_t stream);

/* MLP 16 -> 64 -> 64 -> 3 with GELU (float32): dY (batch x 3) from dX (batch x 16). */
int ipr_mlp_forward(const float* dParams, const float* dX, float* dY, int batch,
                    hipStream_t stream);

/* One training step on a mini-batch: mean squared error against dT (batch x 3),
 * gradient into dGrad (IPR_MLP_NPARAM), then an Adam update of dParams with
 * moments dM, dV (IPR_MLP_NPARAM each) at step `step` (1-based). The batch
 * loss is written to *dLoss (device float). dWork >= ipr_mlp_workspace(batch). */
int ipr_mlp_train_step(float* dParams, float* dGrad, float* dM, float* dV, const float* dX,
                       const float* dT, int batch, int step, float lr, float* dLoss,
                       void* dWork, size_t work_bytes, hipStream_t stream);
size_t ipr_mlp_workspace(int batch);

/* Iteration counts of eq. (1) in exact arithmetic, per eigenvalue (the
 * training labels of the learned start): for matrix i with eigenvalues
 * dLam[offsets[i] .. offsets[i] + n[i]) (device, n[i] <= 2048), root p[i],
 * scale scale[i] (host; s = sqrt(||A||_1 ||A||_inf)) and candidate start c
 * (host cand[3c .. 3c+2] = b0, b1, b2 of C_0 = s^{-1/p} q(A/s)), counts the
 * updates of the coupled iteration until the Frobenius residual is below tol;
 * max_iter + 1 means not reached. counts: host, batch x ncand. With ncand = 0,
 * cand holds one candidate per matrix (batch x 3) and counts has batch entries. */
int ipr_spectral_counts(const double* dLam, const int64_t* offsets, const int* n, const int* p,
                        const double* scale, int batch, const double* cand, int ncand, double tol,
                        int max_iter, int* counts, void* dWork, size_t work_bytes,
                        hipStream_t stream);

/* Message describing the last error of the calling thread ("" if none). */
const char* ipr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IPR_H */
