/*
 * qrcp.h -- C ABI of the MI355X (gfx950) blocked randomized QR with column
 * pivoting (BQRRP, arXiv 2507.00976) and of its unpivoted Householder QR
 * baseline.
 *
 * Conventions for every entry point:
 *  - Matrices are FP64, column-major (LAPACK layout) with an explicit leading
 *    dimension.  Pointers documented as DEVICE point to GPU memory owned by the
 *    caller; HOST pointers to ordinary host memory.  The library never frees or
 *    keeps a caller pointer beyond the call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    All device work is enqueued on it.  The blocking calls return after the
 *    stream has drained the call's work.
 *  - Workspace: the caller passes a DEVICE buffer of at least the size
 *    reported by the matching *_workspace_size() query; nothing is allocated
 *    inside the factorization calls.
 *  - Return value: 0 on success; -i when the i-th argument is illegal (checked
 *    on the host before any launch, LAPACK style); a positive QRCP_ERR_* code
 *    otherwise.  qrcp_status_string() names every code.
 *  - Indices are 0-based unless a call says otherwise (the paper's notation,
 *    Sec. 1.3; LAPACK's one-based pivots on request).
 */
#ifndef QRCP_H
#define QRCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  QRCP_OK = 0,
  QRCP_ERR_WORKSPACE = 1,   /* workspace missing or smaller than required       */
  QRCP_ERR_HIP = 2,         /* a HIP runtime call or kernel launch failed        */
  QRCP_ERR_NONFINITE = 3,   /* NaN/Inf in the input or in the sketch             */
  QRCP_ERR_UNSUPPORTED = 4, /* valid but not implemented (e.g. d > 1024)         */
  QRCP_ERR_TIMEOUT = 5      /* a cross-workgroup wait exceeded its spin limit     */
};

/* Variant choices of the method (Sec. 3 "Input and output specification":
 * the user picks the subroutines).  Pass NULL for the defaults. */
typedef struct qrcp_opts {
  int32_t struct_size;        /* sizeof(qrcp_opts)                                  */
  int32_t cholqr_passes;      /* 1 = one Cholesky QR pass as in Alg. 3 (default);
                                 2 = Cholesky QR repeated once on Q (CholQR2)        */
  int32_t sketch_precision;   /* 0 = FP64 sketch GEMM (default);
                                 1 = BF16 operands, FP32 accumulation, FP64 result   */
  int32_t trailing_precision; /* 0 = FP64 trailing update (default);
                                 1 = FP32 operands and accumulation, FP64 storage    */
  int32_t pivot_base;         /* 0 (default) or 1: base of the returned jpiv         */
  int32_t pivot_steps;        /* 0 = the full GETRF of each block's sketch, min(d, n_i, m_i)
                                 elimination steps (Alg. 2, default);
                                 1 = only the block's k_max = min(b, n_i, m_i) steps:
                                 the same selected columns (partial pivoting at step j
                                 depends on the steps before j alone), but the columns
                                 that no block selects (the residual block after an
                                 early exit) come out in another order, and R agrees
                                 with the default only to rounding                      */
  int32_t qr_tall;            /* panel QR: 0 = preconditioned Cholesky QR + Householder
                                 reconstruction (Alg. 3, default); 1 = Householder QR
                                 of the panel, GEQRF (Sec. 2.3; m <= 65536)             */
  int32_t qrcp_wide;          /* pivots of the sketch: 0 = LU (Alg. 2, default);
                                 1 = column-norm pivoted QR of the sketch (GEQP3)       */
  int64_t max_rank;           /* 0 = no limit (default); l > 0: truncated output, the
                                 loop stops once l columns are factored (the last block
                                 factors only up to column l); rank <= l and
                                 A(rank:, rank:) holds the residual block               */
} qrcp_opts;

/* Bytes of DEVICE workspace qrcp_factor needs for these sizes and options. */
size_t qrcp_workspace_size(int64_t m, int64_t n, int64_t block_size, double sketch_factor,
                           const qrcp_opts* opts);

/*
 * Blocked randomized QRCP (Alg. 1 with the LU-based wide QRCP of Alg. 2 and
 * the preconditioned Cholesky QR + Householder reconstruction of Alg. 3).
 *
 *  A       DEVICE in/out, m x n, lda >= max(1,m).  On return (GEQP3 format,
 *          Sec. 1.3): R (rank x n, upper trapezoidal) on and above the
 *          diagonal, the Householder vectors (implicit unit head) below it for
 *          the first `rank` columns, and the residual block A(rank:, rank:)
 *          when rank < n.
 *  m, n    >= 0, any aspect ratio (Sec. 1.3): for m < n the loop ends after
 *          the block that reaches row m and R is m x n upper trapezoidal.
 *  block_size   b >= 1.
 *  sketch_factor gamma >= 1; the sketch has d = ceil(gamma*b) rows
 *          (d <= 1024 and n <= 32768, else QRCP_ERR_UNSUPPORTED, returned
 *          before any launch: the pivot selection keeps the n_i x d
 *          transposed sketch in at most 256 resident workgroups of 128 rows).
 *  seed    key of the Philox4x32-10 stream that draws the Gaussian sketching
 *          operator (Sec. 2: randomness is used once, before the loop).
 *  tol     >= 0; block rank = leading run of |Rsk(t,t)| > tol * (largest
 *          column norm of the initial sketch) (Sec. 2.2).  0 stops only on
 *          exact zeros.
 *  jpiv    DEVICE out, n int64: column t of A P is column jpiv[t] of A.
 *  tau     DEVICE out, min(m,n) doubles: reflector scalars, 0 beyond rank.
 *  rank    HOST out: the detected rank l.
 *  opts    NULL = defaults.
 *  workspace, workspace_bytes  DEVICE scratch, >= qrcp_workspace_size().
 * Rank deficiency is not an error.  QRCP_ERR_NONFINITE leaves A partially
 * factored.
 */
int qrcp_factor(double* A, int64_t m, int64_t n, int64_t lda, int64_t block_size,
                double sketch_factor, uint64_t seed, double tol, int64_t* jpiv, double* tau,
                int64_t* rank, const qrcp_opts* opts, void* workspace, size_t workspace_bytes,
                void* stream);

/*
 * Stream-ordered form of qrcp_factor (Alg. 1): every block of the loop is
 * enqueued on `stream` without reading anything back (the block's effective
 * width and the stopping decision stay on the device; the launches of the
 * blocks after the stop return at once), and the call returns before the
 * work runs.  Results land in device memory once the stream reaches them:
 * A, jpiv, tau as in qrcp_factor, and
 *  rank_dev    DEVICE out, one int64: the detected rank l;
 *  status_dev  DEVICE out, one int32: QRCP_OK or a QRCP_ERR_* code found on
 *              the device (QRCP_ERR_NONFINITE, QRCP_ERR_TIMEOUT).
 * The return value reports only what the host checks before any launch
 * (illegal arguments -i, QRCP_ERR_UNSUPPORTED, QRCP_ERR_WORKSPACE,
 * QRCP_ERR_HIP); argument numbering follows this signature (rank_dev = -11,
 * status_dev = -12, opts = -13).  The caller keeps A, jpiv, tau, the two
 * result words and the workspace alive until the stream has passed the call.
 * The results equal qrcp_factor's bitwise (qrcp_factor is this call followed
 * by one read-back).  Besides `stream` the call uses the library's second
 * stream of the calling thread for the lookahead, joined into `stream`
 * before the call's last launch.
 */
int qrcp_factor_async(double* A, int64_t m, int64_t n, int64_t lda, int64_t block_size,
                      double sketch_factor, uint64_t seed, double tol, int64_t* jpiv, double* tau,
                      int64_t* rank_dev, int32_t* status_dev, const qrcp_opts* opts,
                      void* workspace, size_t workspace_bytes, void* stream);

/*
 * qrcp_factor without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts that
 * forbid hipMalloc).  The workspace is a fixed device array inside the library
 * (qrcp_noalloc_max_bytes() bytes, 192 MiB; each GPU that loads the library
 * holds its own copy until the process ends); the call allocates nothing and
 * creates no stream: every launch goes to `stream`, in qrcp_factor's order,
 * with the same kernels, so the results equal qrcp_factor's bitwise.
 * Arguments, outputs and errors as qrcp_factor; sizes whose
 * qrcp_workspace_size() exceeds the array return QRCP_ERR_WORKSPACE before any
 * launch (e.g. m = 4096, n = 1024, b = 64 needs 159 MiB and fits; 4096 x 4096
 * at b = 256 does not).  All calls on one GPU share its array: calls that
 * overlap in time on one GPU (two host threads, or two streams) race and give
 * undefined results; serialize them.
 */
size_t qrcp_noalloc_max_bytes(void);
int qrcp_factor_noalloc(double* A, int64_t m, int64_t n, int64_t lda, int64_t block_size,
                        double sketch_factor, uint64_t seed, double tol, int64_t* jpiv,
                        double* tau, int64_t* rank, const qrcp_opts* opts, void* stream);

/* Unpivoted blocked Householder QR (GEQRF format), the performance baseline
 * the canonical FLOP rate is compared against (Sec. 1.4, Sec. 7).  A is m x n
 * DEVICE (m >= n), tau DEVICE min(m,n), nb = panel width. */
size_t qrcp_geqrf_workspace_size(int64_t m, int64_t n, int64_t nb);
int qrcp_geqrf(double* A, int64_t m, int64_t n, int64_t lda, double* tau, int64_t nb,
               void* workspace, size_t workspace_bytes, void* stream);

const char* qrcp_status_string(int status);
/* Text of the last HIP error seen by the calling thread ("" if none). */
const char* qrcp_last_error(void);

/* ------------------------------------------------------------------------
 * Step entry points: each runs one step of the per-block loop with the same
 * kernels qrcp_factor uses, so every step can be checked on its own.
 * ---------------------------------------------------------------------- */

/* S (d x m, N(0,1) entries) stored transposed: St is m x d, ld = ldst >= m.
 * Entry S(2p, j), S(2p+1, j) = Box-Muller pair of Philox4x32-10 block
 * counter (j, p, 0, 0), key (seed lo32, seed hi32):
 *   u1 = (2*(w01 >> 12) + 1) 2^-53,  u2 = (w23 >> 11) 2^-53,
 *   S(2p,j) = sqrt(-2 ln u1) cos(2 pi u2), S(2p+1,j) = sqrt(-2 ln u1) sin(2 pi u2)
 * (Alg. 1 sampling step; Sec. 3 "Initial sketching details"). */
int qrcp_sketch_operator(double* St, int64_t m, int64_t d, int64_t ldst, uint64_t seed,
                         void* stream);
/* Raw Philox4x32-10 blocks: ctr DEVICE count x 4 uint32, out DEVICE count x 4. */
int qrcp_philox(const uint32_t* ctr, int64_t count, uint32_t key0, uint32_t key1, uint32_t* out,
                void* stream);
/* M^sk = S A (Alg. 1 sketching step).  A DEVICE m x n (lda), Msk DEVICE d x n
 * (ldmsk >= d).  precision: 0 FP64, 1 BF16 operands with FP32 accumulation.
 * workspace >= m*d*8 + 40 MiB + 512 bytes (S^T, then split-K partials of
 * the product); less gives QRCP_ERR_WORKSPACE. */
int qrcp_sketch(const double* A, int64_t m, int64_t n, int64_t lda, int64_t d, uint64_t seed,
                int32_t precision, double* Msk, int64_t ldmsk, void* workspace,
                size_t workspace_bytes, void* stream);

/* Pivots of a wide sketch by GETRF on its transpose (Alg. 2).  Msk DEVICE
 * d x ni (ld >= d), read only.  Outputs (DEVICE): ipiv[min(d,ni)] in LAPACK
 * swap format (0-based positions), jsk[ni] the converted permutation (column t
 * of the permuted sketch is column jsk[t]).  Ties in |pivot| go to the
 * smallest current position.  workspace >= qrcp_lu_workspace_size(). */
size_t qrcp_lu_workspace_size(int64_t d, int64_t ni);
int qrcp_lu_pivots(const double* Msk, int64_t d, int64_t ni, int64_t ldmsk, int64_t* ipiv,
                   int64_t* jsk, void* workspace, size_t workspace_bytes, void* stream);

/* GEQRF of a permuted wide sketch (Alg. 2 last step): B DEVICE d x ni (ld >=
 * d) holding the columns in pivot order, read only; R DEVICE d x ni (ldr >= d)
 * receives the upper trapezoidal R (exact zeros below the diagonal). */
size_t qrcp_sketch_qr_workspace_size(int64_t d, int64_t ni);
int qrcp_sketch_qr(const double* B, int64_t d, int64_t ni, int64_t ldb, double* R, int64_t ldr,
                   void* workspace, size_t workspace_bytes, void* stream);

/* Preconditioned Cholesky QR of a panel (Alg. 3 first two steps):
 * P DEVICE mi x k (ldp) is overwritten by Q = P Rs^{-1} Rc^{-1}, Rs DEVICE k x k
 * upper (ldrs), Rc DEVICE k x k (ldrc) receives the Cholesky factor, *keff
 * (HOST) the number of columns factored before a Cholesky breakdown (== k when
 * none).  passes = 1 or 2.  workspace >= qrcp_panel_workspace_size(). */
size_t qrcp_panel_workspace_size(int64_t mi, int64_t k);
int qrcp_cholqr(double* P, int64_t mi, int64_t k, int64_t ldp, const double* Rs, int64_t ldrs,
                double* Rc, int64_t ldrc, int32_t passes, int64_t* keff, void* workspace,
                size_t workspace_bytes, void* stream);

/* Householder reconstruction of an orthonormal Q (Alg. 3 third step, after
 * Ballard et al.'s modified LU): Q DEVICE mi x k (ldq) is overwritten by Y
 * (strictly below the diagonal; the unit diagonal is implicit) and U on and
 * above it; tau DEVICE k, dsig DEVICE k (the sign vector D).  The first k
 * columns of H_0 ... H_{k-1} equal Q diag(D). */
int qrcp_reconstruct(double* Q, int64_t mi, int64_t k, int64_t ldq, double* tau, double* dsig,
                     void* workspace, size_t workspace_bytes, void* stream);

/* C <- (H_0 ... H_{k-1})^T C (ORMQR left/transpose, Sec. 2.4) with Y DEVICE
 * mi x k (unit lower trapezoidal read from below the diagonal, ldy), tau DEVICE
 * k, C DEVICE mi x nc (ldc).  precision 0 = FP64, 1 = FP32 GEMMs. */
size_t qrcp_apply_qt_workspace_size(int64_t mi, int64_t k, int64_t nc);
int qrcp_apply_qt(const double* Y, int64_t mi, int64_t k, int64_t ldy, const double* tau,
                  double* C, int64_t nc, int64_t ldc, int32_t precision, void* workspace,
                  size_t workspace_bytes, void* stream);

/* Sketch update (Alg. 1 last step, Sec. 3 "Sample update"):
 * Out(0:b, :) = Rsk12 - Rsk11 R11^{-1} R12 and Out(b:d, :) = Rsk22 are formed in
 * place in Rsk: Rsk DEVICE d x (b + nt) (ld), R11 DEVICE b x b upper (ldr11),
 * R12 DEVICE b x nt (ldr12).  On return Rsk(:, b:b+nt) holds the updated
 * sketch. */
int qrcp_sketch_update(double* Rsk, int64_t d, int64_t b, int64_t nt, int64_t ldrsk,
                       const double* R11, int64_t ldr11, const double* R12, int64_t ldr12,
                       void* workspace, size_t workspace_bytes, void* stream);
/* The same update as qrcp_factor forms it after one Cholesky QR pass
 * (Alg. 3 with R11 = diag(D) Rc Rsk11): Rsk11 R11^{-1} = Rc^{-1} diag(D), so
 *   Out(0:b, :) = Rsk12 - Rc^{-1} diag(D) R12.
 * Rc DEVICE b x b upper (ldrc), dsig DEVICE b (entries +-1), the rest as in
 * qrcp_sketch_update; workspace >= 2 b^2 doubles + 1 KiB. */
int qrcp_sketch_update_chol(double* Rsk, int64_t d, int64_t b, int64_t nt, int64_t ldrsk,
                            const double* Rc, int64_t ldrc, const double* dsig, const double* R12,
                            int64_t ldr12, void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Request server: many independent factorizations of mixed shapes in flight
 * on one GPU (the paper's method applied per request; continuous admission).
 *
 * Worker threads (`slots`, each with its own HIP stream) take requests from
 * one FIFO queue as soon as they can be admitted: the request's workspace
 * fits a free slice of the server's device pool (`hbm_budget` bytes, carved
 * once at creation; a slice goes back to the pool when its request
 * completes, so nothing is allocated or freed while requests run), and the
 * cross-workgroup-waiting kernels of the running requests fit the device's
 * compute units together.  Requests that arrive while others run start as
 * soon as a slot and memory free up; their kernels overlap on the device.
 * A request computes exactly what qrcp_factor computes on the same arguments
 * (bitwise: the same kernels in the same order; a worker runs all of them on
 * its own stream, without qrcp_factor's second stream for the deferred
 * update, since the concurrent requests already fill the device).
 * ---------------------------------------------------------------------- */
typedef struct qrcp_server qrcp_server;

typedef struct qrcp_server_cfg {
  int32_t struct_size; /* sizeof(qrcp_server_cfg)                                */
  int32_t slots;       /* worker threads / streams, 1..64 (0 = 8)                  */
  int64_t hbm_budget;  /* bytes of the device pool allocated at creation (0 = the
                          smaller of 4 GiB and 80% of the free device memory)     */
  int32_t device;      /* HIP device ordinal                                      */
} qrcp_server_cfg;

typedef struct qrcp_request {
  int32_t struct_size;   /* sizeof(qrcp_request)                                  */
  int64_t m, n, lda;     /* as qrcp_factor                                        */
  int64_t block_size;
  double sketch_factor;
  uint64_t seed;
  double tol;
  double* A;             /* DEVICE, caller-owned until the request completes      */
  int64_t* jpiv;         /* DEVICE out, n                                         */
  double* tau;           /* DEVICE out, min(m, n)                                 */
  qrcp_opts opts;        /* struct_size = 0 selects the defaults                  */
} qrcp_request;

typedef struct qrcp_result {
  int32_t struct_size;
  int32_t status;        /* qrcp_factor's return value                            */
  int64_t rank;
  double submit_ms;      /* server clock: ms since qrcp_server_create             */
  double start_ms;       /* admitted and started                                  */
  double end_ms;         /* results final in device memory                        */
} qrcp_result;

/* NULL on failure (bad config, no device). */
qrcp_server* qrcp_server_create(const qrcp_server_cfg* cfg);
/* Queues a request; *ticket identifies it.  -i: i-th argument illegal;
 * QRCP_ERR_UNSUPPORTED if it can never be admitted (workspace above the
 * budget, resident grid above the device). */
int qrcp_server_submit(qrcp_server* s, const qrcp_request* req, uint64_t* ticket);
/* 0 = done (*out filled, ticket released), 1 = pending, -2 = unknown ticket. */
int qrcp_server_poll(qrcp_server* s, uint64_t ticket, qrcp_result* out);
/* Blocks until the request is done; 0, or -2 for an unknown ticket. */
int qrcp_server_wait(qrcp_server* s, uint64_t ticket, qrcp_result* out);
/* Requests submitted and not yet done. */
int qrcp_server_pending(qrcp_server* s);
/* Finishes every queued request, then frees the server. */
void qrcp_server_destroy(qrcp_server* s);

/* ------------------------------------------------------------------------
 * Stage timing (instrumentation, not part of the method).  mode 0 = off,
 * 1 = time only the trailing-update product C += Y W2 (the dominant kernel),
 * 2 = time every stage of the loop.  Enabling clears earlier records.  HIP
 * events are recorded on the stream of each call; qrcp_profile_read() waits
 * for them and returns the summed device time (ms), the number of timed
 * launches and the algorithmic flops attributed to the stage.  Not thread
 * safe: one profiling client per process.
 * ---------------------------------------------------------------------- */
int qrcp_profile_enable(int32_t mode);
int32_t qrcp_profile_num_stages(void);
const char* qrcp_profile_stage_name(int32_t stage);
int qrcp_profile_read(int32_t stage, double* ms, int64_t* count, double* flops);

#ifdef __cplusplus
}
#endif

#endif /* QRCP_H */
