/*
 * cscirc.h -- C ABI of the MI355X (gfx950) partial-circulant LASSO library.
 *
 * Problem (Fiandrotti, Fosson, Ravazzi, Magli, arXiv 1707.02244):
 *   measurements y = A x* with A = P C (Eq. 1; Section 4.3), where
 *     C (n x n) is circulant with first column c:  C[i][j] = c[(i - j) mod n]
 *     P (m x n) keeps rows 0, d, 2d, ..., (m-1)d:   A[r][j] = c[(r*d - j) mod n]
 *   and recovery solves the LASSO (Eq. 3, halved)
 *     min_x 1/2 ||y - A x||^2 + lambda ||x||_1
 *   with ISTA (Alg. 1) or ADMM (Alg. 2).
 *
 * Conventions for every call:
 *   - Every float pointer is a DEVICE pointer on the current HIP device,
 *     float32, densely packed, owned by the caller.  The library never frees
 *     or retains it beyond the work it enqueues.
 *   - n is a power of two with 64 <= n <= 2^26; d is 1, 2, 4, 8 or 16 with
 *     d <= n; m = n/d.  d = 1 (A = C, every row kept), n < 256 and n > 2^22
 *     run the two-launch schedule; the direct products take d >= 2 and
 *     n >= 256, the unrolled solver d >= 2 and n <= 2^25.
 *   - All work is enqueued on `stream` (a hipStream_t; 0 is the null stream)
 *     and the call returns without synchronising.  Outputs are valid once the
 *     stream has been synchronised.
 *   - Arguments are validated on the host before anything is enqueued; a bad
 *     argument returns CS_EINVAL and enqueues nothing.  cs_last_error() gives
 *     a message (per thread).
 *   - The first call for a given (device, n, d) builds a plan: twiddle tables
 *     (double precision on the host) and a workspace of about 3*n*4 bytes,
 *     allocated with hipMalloc and kept until the process ends (or the
 *     caller's block, see cs_set_workspace).  Calls that share a plan share
 *     its workspace: issue them on one stream (or serialise them);
 *     concurrent calls with the same (n, d) on different streams race.
 *   - No C++ exception crosses this interface.
 */
#ifndef CSCIRC_H
#define CSCIRC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CS_OK = 0,
  CS_EINVAL = -1,   /* invalid argument (checked before any work is enqueued) */
  CS_ENOMEM = -2,   /* device allocation for a plan failed                    */
  CS_EHIP = -3,     /* a HIP runtime call or kernel launch reported an error  */
  CS_ENOTSUP = -4   /* a valid but unsupported request                        */
} cs_status;

typedef struct ihipStream_t* cs_stream; /* hipStream_t */

/* y = A x = P C x  (Eq. 1).  c: n, x: n, y: m.  */
cs_status cs_circ_apply(const float* c, int64_t n, int32_t d, const float* x, float* y,
                        cs_stream stream);

/* x = A^T r = C^T P^T r  (the transpose product of Alg. 1, step 4).
 * c: n, r: m, x: n.  */
cs_status cs_circ_apply_T(const float* c, int64_t n, int32_t d, const float* r, float* x,
                          cs_stream stream);

/* The same two products evaluated directly, without the FFT: every output
 * is an inner product over the generator c, as in the paper's GPU kernels
 * (Section 4: the CPISTA residual kernel takes a row of A times x, the
 * thresholded-gradient kernel a row of A^T times r, reading only c):
 *     y_i = sum_{j<n} c[(d i - j) mod n] x_j   (i < m),
 *     x_j = sum_{i<m} c[(d i - j) mod n] r_i   (j < n).
 * Arguments, layouts, ownership and errors as cs_circ_apply /
 * cs_circ_apply_T (device pointers; c: n, x: n, y: m, r: m; no allocation).
 * O(n m) work with FP32 accumulation in input order: a baseline that shows
 * what the FFT formulation buys over direct inner products, not a solver
 * path.  */
cs_status cs_circ_apply_direct(const float* c, int64_t n, int32_t d, const float* x, float* y,
                               cs_stream stream);
cs_status cs_circ_apply_T_direct(const float* c, int64_t n, int32_t d, const float* r, float* x,
                                 cs_stream stream);

/* max_k |c_hat_k|^2 over the n-point DFT of c, written to out[0] (device).
 * It bounds ||A||_2^2 from above, so tau = 1/out is an admissible ISTA step
 * (Alg. 1 asks for tau in (0, ||A||_2^-2)).  */
cs_status cs_circ_norm_bound(const float* c, int64_t n, float* out, cs_stream stream);

/* Generator of the composite circulant C B of the compressed-deblurring
 * problem (Section 7): B is the order-L box blur, the circulant whose rows
 * are right-circular shifts of b with b_j = 1/L for j < L and 0 otherwise,
 * and C B is again circulant (a product of circulants), with first column
 *     out[k] = (1/L) sum_{t<L} c[(k + t) mod n],   k < n,
 * each sum taken in double and rounded once to float.  Pass `out` as the
 * generator of any call above to solve with A = P C B.
 * c: n device floats, out: n device floats (distinct from c); n a power of
 * two in [2^6, 2^26] (the solvers' range); 1 <= L <= min(n, 4096) (O(n L)
 * work).  No allocation; CS_EINVAL on a bad argument, nothing enqueued.  */
cs_status cs_box_blur_generator(const float* c, int64_t n, int32_t L, float* out, cs_stream stream);

/* ISTA, Alg. 1:  x(0) = 0;  for t = 1..iters:
 *     x(t) = eta_{tau*lambda}( x(t-1) + tau A^T (y - A x(t-1)) )
 * eta is the soft threshold of Eq. 4 (strict comparison).  The threshold is
 * tau*lambda (proximal-gradient reading of the LASSO of Eq. 3 with alpha =
 * lambda).  y: m.  x: n, output x(iters) (zero when iters == 0).
 * obj: NULL, or a device array of `iters` floats that receives the LASSO
 * objective of Eq. 3 (halved) along the iterates,
 *     obj[t-1] = F(x(t)) = 1/2 ||y - A x(t)||^2 + lambda ||x(t)||_1,
 * the residual taken by Parseval from the m-point spectrum the iteration
 * already forms and summed in double per workgroup.  A trace keeps the
 * schedule an untraced call takes (the persistent single launch where it
 * applies, see cs_set_solver_path); the iterates are the same with or
 * without it.
 * Requires lambda >= 0, tau > 0, iters >= 0.  */
cs_status cs_ista_solve(const float* c, int64_t n, int32_t d, const float* y, float lambda,
                        float tau, int32_t iters, float* x, float* obj, cs_stream stream);

/* ADMM, Alg. 2 (scaled dual u):  for t = 1..iters:
 *     x(t) = (A^T A + rho I)^{-1} (A^T y + rho (z(t-1) - u(t-1)))
 *     z(t) = eta_{lambda/rho}( x(t) + u(t-1) )
 *     u(t) = u(t-1) + x(t) - z(t)
 * The inverse is applied exactly through the Woodbury identity with the
 * m x m circulant A A^T (never formed).  warm == 0: start from
 * x = z = u = 0 (Alg. 2's initial guess); warm != 0: start from the z and u
 * passed in.  x, z, u: n each, outputs x(iters), z(iters), u(iters); u is
 * also used as the dual state during the solve.  With iters == 0 and warm ==
 * 0 all three are zeroed; with warm != 0 they are left as passed.
 * obj: NULL, or a device array of `iters` floats that receives
 *     obj[t-1] = F(x(t)) = 1/2 ||y - A x(t)||^2 + lambda ||x(t)||_1
 * for the x-update iterate (Eq. 3 halved; the same Parseval residual as
 * ISTA's), on the same schedule as an untraced call.
 * Requires lambda >= 0, rho > 0, iters >= 0.  */
cs_status cs_admm_solve(const float* c, int64_t n, int32_t d, const float* y, float lambda,
                        float rho, int32_t iters, int32_t warm, float* x, float* z, float* u,
                        float* obj, cs_stream stream);

/* Batched ISTA (Alg. 1) over `count` independent signals of different
 * lengths and decimations, in one persistent launch.
 *
 * Signal i has length n_host[i] (a power of two in [2^10, 2^18]) and
 * decimation d_host[i] (2, 4 or 8; m_i = n_i / d_i); its generator is
 * c_cat[off_n_host[i] .. + n_i), its measurements y_cat[off_m_host[i] .. +
 * m_i), its parameters lambda_dev[i] and tau_dev[i] (device arrays of `count`
 * floats, lambda >= 0, tau > 0) and its output x_cat[off_n_host[i] .. + n_i).
 * n_host, d_host and the offsets are HOST arrays; off_n must be even and the
 * n-length output slices must not overlap (CS_EINVAL otherwise).  Each signal
 * is solved with the arithmetic of cs_ista_solve, from x(0) = 0, for `iters`
 * iterations (iters == 0 writes x = 0).
 *
 * The whole batch is one cooperative launch: every workgroup owns row and
 * column items of one size class (length and decimation) for the whole
 * solve, and all signals advance together, one grid barrier after each pass.
 * A plan per batch shape (device, lengths, decimations, offsets) holds the
 * spectra and tables of every signal (about 12 n_i bytes each), allocated on
 * the first call and kept (the four most recently used plans are kept).  On
 * that first call a tuner times the candidate schedules (workgroups per CU;
 * the cost model that shares workgroups among size classes) with a few
 * iterations into a temporary block (the caller's outputs are not written),
 * synchronising the stream; if the environment variable CSCIRC_TUNE_CACHE
 * names a file, choices are read from and appended to it.  The launch is
 * recorded in a HIP graph once per (plan, iters) and replayed.  A change of
 * device pointers since the previous call uploads the signal descriptors
 * with a synchronous copy.  Batched calls on one device must be serialised.
 * A barrier wait that exceeds its bound is reported by cs_check_device.  */
cs_status cs_ista_solve_batched(int32_t count, const int64_t* n_host, const int32_t* d_host,
                                const int64_t* off_n_host, const int64_t* off_m_host, const float* c_cat,
                                const float* y_cat, const float* lambda_dev, const float* tau_dev, int32_t iters,
                                float* x_cat, cs_stream stream);

/* Batched ADMM (Alg. 2, the x-update by Woodbury as in cs_admm_solve) over
 * independent signals, in one persistent launch, with the same batch layout,
 * plan, tuner and graph as cs_ista_solve_batched.  Per signal: lambda_dev[i]
 * >= 0 and rho_dev[i] > 0 (device arrays); outputs x, z, u (n_i each) at
 * off_n_host[i] of x_cat, z_cat, u_cat.  warm == 0 starts from x = z = u = 0
 * (Alg. 2's initial guess); warm != 0 starts from the z and u passed in.
 * iters == 0: cold writes x = z = u = 0, warm leaves them as passed.  */
cs_status cs_admm_solve_batched(int32_t count, const int64_t* n_host, const int32_t* d_host,
                                const int64_t* off_n_host, const int64_t* off_m_host, const float* c_cat,
                                const float* y_cat, const float* lambda_dev, const float* rho_dev, int32_t iters,
                                int32_t warm, float* x_cat, float* z_cat, float* u_cat, cs_stream stream);

/* The schedule of the last batched call as a JSON object (grid, workgroups
 * per CU, cost model, whether a graph was replayed, the shape key and the
 * tuner's trials with their times), copied into buf (cap bytes, NUL
 * included).  CS_EINVAL if buf is NULL or too small.  */
cs_status cs_batched_schedule(char* buf, size_t cap);

/* Differentiable unrolled ISTA (Alg. 1 with learnable per-iteration
 * parameters) over a batch of Bt signals that share one operator A = P C:
 *     x_0 = 0,  v_t = x_{t-1} + tau[t] A^T (y_b - A x_{t-1}),
 *     x_t = eta_{tau[t] lam[t]}(v_t),   t = 1..K  (0-based arrays).
 * lam and tau are DEVICE arrays of K floats; y is Bt x m row-major; xK is
 * Bt x n.  The forward pass stores x at t = every, 2 every, ... (< K) in the
 * caller's checkpoint area of cs_unrolled_ckpt_bytes() bytes.  The backward
 * pass takes g_xK = dL/dx_K (Bt x n), recomputes each segment of `every`
 * steps from its checkpoint and runs the adjoint of the recursion, writing
 * g_lam (K), g_tau (K) and g_y (Bt x m), all device arrays.  The threshold's
 * derivative is taken as 0 where |v_t| equals the threshold.  A workspace per
 * (device, n, d, Bt, every) is allocated on first use (about
 * (3 + 2 every) Bt n floats plus 3 Bt n/2 complex) and kept.  */
size_t cs_unrolled_ckpt_bytes(int64_t n, int32_t d, int32_t Bt, int32_t K, int32_t every);
cs_status cs_unrolled_ista_fwd(const float* c, int64_t n, int32_t d, int32_t Bt, const float* y, const float* lam,
                               const float* tau, int32_t K, int32_t every, float* xK, void* ckpt,
                               cs_stream stream);
cs_status cs_unrolled_ista_bwd(const float* c, int64_t n, int32_t d, int32_t Bt, const float* y, const float* lam,
                               const float* tau, int32_t K, int32_t every, const void* ckpt, const float* g_xK,
                               float* g_lam, float* g_tau, float* g_y, cs_stream stream);

/* ---- 2-D sensing with a blur --------------------------------------------
 * An image x of `rows` x `cols` pixels (row-major; both powers of two,
 * 16 <= rows <= 8192, 16 <= cols <= 4096) is blurred by a point-spread
 * function h and sensed by a 2-D kernel s, both by periodic 2-D convolution
 * ((K x)[i][j] = sum_{a,b} k[(i-a) mod rows][(j-b) mod cols] x[a][b]), then
 * decimated to the pixels (2i, 2j):
 *     y = A x = P C H x,   y: rows/2 x cols/2 (row-major).
 * The blur as one more circulant factor is how Section 7 casts deblurring;
 * C H is doubly block circulant, so the 2-D DFT diagonalises it with
 * eigenvalues DFT2(s) * DFT2(h), and A A^T is the (rows/2 x cols/2) doubly
 * block circulant with eigenvalues the 2x2 alias averages of their squared
 * magnitudes.  s and h are rows x cols device arrays; h may be NULL (no
 * blur).  The decimation is 2 along both axes.  A plan per (device, rows,
 * cols) holds about 2.5 rows*cols complex values of workspace (kept), and
 * every call recomputes DFT2(s) DFT2(h) and (solvers) DFT2(y) on the
 * stream.  Same conventions as above otherwise.  */
cs_status cs2_apply(const float* s, const float* h, int32_t rows, int32_t cols, const float* x, float* y,
                    cs_stream stream);
/* x = A^T r = H^T C^T P^T r.  r: rows/2 x cols/2, x: rows x cols.  */
cs_status cs2_apply_T(const float* s, const float* h, int32_t rows, int32_t cols, const float* r, float* x,
                      cs_stream stream);
/* max |DFT2(s) DFT2(h)|^2 written to out[0] (device): an upper bound on
 * ||A||_2^2, so tau = 1/out is an admissible ISTA step.  */
cs_status cs2_norm_bound(const float* s, const float* h, int32_t rows, int32_t cols, float* out,
                         cs_stream stream);
/* ISTA (Alg. 1) on the 2-D operator, as cs_ista_solve: x(0) = 0,
 * x(t) = eta_{tau lambda}(x(t-1) + tau A^T (y - A x(t-1))).  x: rows x cols
 * output; obj: NULL or `iters` floats, obj[t-1] = F(x(t)).  */
cs_status cs2_ista_solve(const float* s, const float* h, int32_t rows, int32_t cols, const float* y, float lambda,
                         float tau, int32_t iters, float* x, float* obj, cs_stream stream);
/* ADMM (Alg. 2) on the 2-D operator, as cs_admm_solve (same x, z, u, warm
 * and obj semantics).  The x-update applies (A^T A + rho I)^{-1} exactly in
 * the Fourier domain, in the residual form
 *     X' = W + conj(g_hat) (Y_hat - S_W) / (rho + Lam),
 * W = DFT2(z - u), S_W the 2x2-folded g_hat W: equal to the Woodbury
 * form, but without its cancellation when Lam >> rho.  */
cs_status cs2_admm_solve(const float* s, const float* h, int32_t rows, int32_t cols, const float* y, float lambda,
                         float rho, int32_t iters, int32_t warm, float* x, float* z, float* u, float* obj,
                         cs_stream stream);

/* ---- caller-provided workspace -------------------------------------------
 * The single-signal calls (cs_circ_apply, cs_circ_apply_T, cs_circ_norm_bound,
 * cs_ista_solve, cs_admm_solve) need, per (n, d), one block of device memory:
 * the spectrum buffer of the four-step transform (Section 4.2 diagonalises
 * the circulant with the DFT; the block holds that DFT's intermediate), the
 * tables of c_hat and of the spectrum of P^T y, the twiddle factors and the
 * persistent solver's barrier counters and error flag.  By default the
 * library allocates it on the first call for (device, n, d) and keeps it.
 *
 * cs_workspace_bytes: bytes of that block for (n, d); mode 0 (operators),
 * 1 (ISTA) and 2 (ADMM) share one layout.  Returns 0 for an invalid n, d or
 * mode.
 *
 * cs_set_workspace: from now on the single-signal calls on the current
 * device use the caller's block `ws` (a DEVICE pointer, 256-byte aligned,
 * `bytes` long, owned by the caller) instead of library memory: a call whose
 * (n, d) needs more than `bytes` returns CS_EINVAL and enqueues nothing.  The
 * library writes the twiddle tables into the block with a kernel on the
 * call's stream whenever a call's n differs from the previous call's, and
 * clears the barrier area on the block's first use; the caller must not
 * modify the block while it is set.  Calls that use one block race unless
 * they are issued on one stream.  ws == NULL returns to library memory.  An
 * objective trace (obj != NULL) still takes a small library buffer of
 * partial sums.  The batched, unrolled and 2-D calls keep their own memory.
 * Errors: CS_EINVAL (misaligned or too small), CS_ENOTSUP (device index of
 * 64 or more).  */
size_t cs_workspace_bytes(int64_t n, int32_t d, int32_t mode);
cs_status cs_set_workspace(void* ws, size_t bytes);

/* Circulant ADMM with an arbitrary row set (Section 4.3, Alg. 3).  A = P C
 * with C the circulant of first column c (n, device) and P keeping the m rows
 * listed in omega_host (a HOST array of m distinct indices in [0, n), any
 * order); y (m, device) holds the measurements in omega's order.  The split
 *     min 1/2 ||y - P v||^2 + alpha ||z||_1   s.t.  v = C x,  z = x
 * is solved from x = v = z = mu = nu = 0 with, per iteration,
 *     x  = (rho C^T C + sigma I)^-1 (rho C^T (v + mu) + sigma (z - nu))
 *     v  = (P^T P + rho I)^-1 (rho C x - rho mu + P^T y)
 *     z  = eta_{alpha/sigma}(x + nu)          (soft threshold, Eq. 4)
 *     mu = mu + tau (v - C x),   nu = nu + tau (x - z)
 * (the updates of the section's augmented Lagrangian; the printed algorithm's
 * "v = v + mu" is read as forming v + mu for the x-update, and one step tau
 * serves both multipliers).  The circulant inverse and C x are applied in the
 * Fourier domain, the diagonal (P^T P + rho I)^-1 in the time domain.
 * Outputs x, v, z, mu, nu (n each, device) after `iters` iterations (all
 * zero for iters == 0).  Requires n a power of two in [2^8, 2^22], 1 <= m <=
 * n, alpha >= 0, rho > 0, sigma > 0, tau > 0 (the section quotes tau <
 * (1 + sqrt 5)/2 for convergence), iters >= 0; CS_EINVAL otherwise,
 * including a repeated or out-of-range index in omega.  Uses the (n, d = 2)
 * plan of the single-signal calls for its c_hat table and twiddles, and a
 * working buffer of the library (24 n bytes: both signals' spectra and the
 * column-blocked mu, nu, P^T y and indicator of omega), allocated with
 * hipMalloc on the first call of a larger n on a device and kept until the
 * process ends; calls on one device share it (serialise them).  omega's
 * indices are copied through x: the call synchronises the stream once, after
 * that copy.  The last iteration writes x, v, z, mu and nu.  Two launches
 * per iteration.  */
cs_status cs_cpadmm_solve(const float* c, int64_t n, const int64_t* omega_host, int64_t m, const float* y,
                          float alpha, float rho, float sigma, float tau, int32_t iters, float* x, float* v,
                          float* z, float* mu, float* nu, cs_stream stream);

/* Allocation-free ISTA, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, arithmetic and results as cs_ista_solve with
 * obj == NULL, for n <= 2^20 (larger n: CS_EINVAL, nothing enqueued).  The
 * plan block (spectrum buffer, c_hat / y_hat tables, twiddles, barrier area;
 * cs_workspace_bytes(2^20, d, 1) = 12.1 MiB) is a static device array of the
 * library, one copy per GPU, held until the process ends; the call itself
 * makes no device allocation.  The array keeps the last call's contents (the
 * library rewrites what a call needs: twiddles when n changes, the barrier
 * counters every call).  All calls on one GPU share the array: calls that
 * overlap on one GPU (other streams, other threads) race; serialise them.
 * The first call on a device looks the array's device address up with
 * hipGetSymbolAddress (CS_EHIP if that fails).  */
cs_status cs_ista_solve_noalloc(const float* c, int64_t n, int32_t d, const float* y, float lambda, float tau,
                                int32_t iters, float* x, cs_stream stream);

/* Solver schedule.  For 2^8 <= n <= 2^22 and d >= 2 a solve runs as ONE
 * cooperative launch, with or without an objective trace: all iterations in
 * a persistent kernel whose workgroups keep the time-domain state in
 * registers and meet at a grid barrier between the row and column passes.
 * Other sizes, d = 1 (or path 1) use two launches per iteration with the
 * state in HBM.  Both compute the same iterates.  path: 0 = choose per size
 * (default), 1 = two launches per iteration, 2 = persistent (the solve
 * returns CS_ENOTSUP where it does not apply).  Process-wide.  */
cs_status cs_set_solver_path(int32_t path);

/* Synchronise `stream` and report device-side errors of earlier solves on
 * the current device: CS_EHIP if a persistent solve's grid-barrier wait hit
 * its bound (its results are then invalid).  Clears the flag.  */
cs_status cs_check_device(cs_stream stream);

/* Kernel timing (diagnostics, for benchmarks).  While enabled, every launch
 * of the solvers' per-iteration kernels (or persistent solve kernel) is bracketed by a pair of
 * hipEvents recorded on the caller's stream.  cs_timing_read waits for the
 * recorded launches of one kernel ("passA_ista", "passB_ista", "passA_admm",
 * "passB_admm", the persistent "solve_ista", "solve_admm", the batched
 * "batch_ista", the direct products "direct", "direct_T", or the 2-D
 * "col2_ista", "row2_ista", "col2_admm",
 * "row2_admm"), returns their count and summed duration in milliseconds,
 * and forgets them.  Timing adds event records to the stream; leave it off
 * for production runs.  */
cs_status cs_timing_enable(int32_t on);
cs_status cs_timing_read(const char* kernel, int64_t* launches, double* total_ms);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* cs_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int32_t cs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CSCIRC_H */
