/*
 * lindblad.h -- C ABI of the MI355X (gfx950) library that turns a GKSL master
 * equation into the real linear ODE dv/dt = Q v + K over the generalized
 * Gell-Mann basis and integrates it with classic fourth-order Runge-Kutta.
 *
 * Method: Meyerov, Kozinov, Liniov, Volokitin, Yusipov, Ivanchenko, Denisov,
 * "Transforming Lindblad Equations into Systems of Real-Valued Linear
 * Equations: Performance Optimization and Parallelization of an Algorithm",
 * arXiv:1912.01491. Equation numbers count the displayed equations of
 * Sections 2-3 in order: (1)-(2) the Lindbladian and its dissipator,
 * (3)-(5) the S, J, D generators, (6) expansion of a Hermitian matrix,
 * (7) the coherence vector, (10) the real ODE, (11) f and d, (12) z,
 * (13) q, (14) k, (15) r. "Table 1" is the paper's algorithm table.
 *
 * Conventions (all entry points):
 *  - N is the Hilbert-space dimension (2 <= N <= LB_MAX_N), M = N*N - 1.
 *  - Basis order, 0-based: S^(j,k) for pairs j<k in row-major pair order
 *    (position j*N - j*(j+1)/2 + k-j-1), then J^(j,k) in the same order
 *    (offset P = N(N-1)/2), then D^1..D^{N-1} (offset 2P). D^l is
 *    (sum_{x<l} e_x e_x^T - l e_l e_l^T) / sqrt(l(l+1)) with 0-based rows,
 *    the Hermitian, trace-orthonormal reading of Eq. (5).
 *  - Complex arrays are interleaved (re, im) doubles, i.e. the layout of
 *    torch.complex128 / numpy complex128. Matrices are row-major.
 *  - Pointers documented "device" are HIP device memory (e.g. torch CUDA
 *    tensors); "host" pointers are ordinary memory. The caller owns every
 *    buffer it passes and keeps it alive until the context stream has
 *    reached the call's completion; the library never frees caller memory.
 *  - Calls that take a context are asynchronous on that context's stream
 *    unless they are documented to return a value to the host (those
 *    synchronize the stream). lb_sync() waits for completion.
 *  - Every function returns LB_OK (0) or a negative status; lb_last_error()
 *    returns a message for the last failure on the calling thread.
 *  - The dissipator is sum_jk gamma_jk (F_j rho F_k - 1/2 {F_k F_j, rho})
 *    with gamma = sum_p g_p l_p l_p^dagger (Eqs. (8), (14), (15)).
 */
#ifndef LINDBLAD_H
#define LINDBLAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_OK 0
#define LB_ERR_INVALID_ARG (-1)   /* null pointer, N out of range, bad sizes, dt not finite, ... */
#define LB_ERR_NOT_HERMITIAN (-2) /* LB_CHECK_HERMITIAN was set and an input is not Hermitian */
#define LB_ERR_OOM (-3)           /* the context workspace could not be allocated */
#define LB_ERR_DEVICE (-4)        /* a HIP call failed; see lb_last_error() */
#define LB_ERR_UNSUPPORTED (-5)   /* valid request the library cannot serve (e.g. too large) */
#define LB_ERR_ADMISSION (-6)     /* a serving request does not fit the server's memory budget */
#define LB_ERR_NO_CONVERGENCE (-7) /* an iterative solve stopped at its iteration limit before its
                                      tolerance; the outputs hold the last iterate */
#define LB_ERR_IO (-8)            /* a file could not be opened, read or written, or is not a valid
                                     saved system (bad header, short, payload hash mismatch) */
#define LB_ERR_CANCELLED (-9)     /* a serving request was still queued when its server was destroyed */

#define LB_MAX_N 2048             /* largest Hilbert-space dimension accepted (dense inputs of that
                                     size would not fit in memory; the sparse path reaches it) */

/* lindblad_prepare flags */
#define LB_CHECK_HERMITIAN 1u     /* verify H and gamma are Hermitian (extra pass, synchronizes) */

/* propagation precision */
#define LB_FP64 0                 /* FP64 storage and arithmetic */
#define LB_FP32 1                 /* Q stored in FP32, FP32 MFMA products, FP64 state and combination */

typedef struct lb_ctx lb_ctx;

/* ------------------------------------------------------------------ */
/* Context                                                            */
/* ------------------------------------------------------------------ */

/* Creates a context on HIP device `device`. `stream` is the hipStream_t the
 * context enqueues on (NULL: the device's default stream). The context owns
 * a device workspace and a pinned host staging buffer that grow on demand
 * and are freed by lb_destroy. A context is not thread-safe; use one per
 * thread. */
int lb_create(lb_ctx** ctx, int device, void* stream);
int lb_destroy(lb_ctx* ctx);
/* Switches the stream subsequent calls are enqueued on (NULL: default stream);
 * waits for the previous stream first. */
int lb_set_stream(lb_ctx* ctx, void* stream);
/* Blocks until all work enqueued through the context has finished. */
int lb_sync(lb_ctx* ctx);
/* Message describing the last failing call on this thread ("" if none). */
const char* lb_last_error(void);
/* Library version, e.g. 100 for 0.1.0. */
int lb_version(void);
/* Progress of long calls (lindblad_spectrum): fn(stage, fraction, user) is
 * called from the calling thread, at most about every two seconds (and when a
 * stage begins or ends), with the
 * stage's name ("hessenberg": columns reduced; "qr": eigenvalues found) and
 * the fraction done in [0, 1]. fn = NULL turns it off (the default). The
 * callback must not call into the library. */
typedef void (*lb_progress_fn)(const char* stage, double fraction, void* user);
int lb_set_progress(lb_ctx* ctx, lb_progress_fn fn, void* user);

/* ------------------------------------------------------------------ */
/* Basis index generator (Sec. 2, Eqs. (3)-(5))                        */
/* ------------------------------------------------------------------ */

/* Host, pure: basis position i -> class (0 = S, 1 = J, 2 = D) and (j, k);
 * for D, *j = l in 1..N-1 and *k = 0. */
int lb_basis_index(int N, int64_t i, int32_t* cls, int32_t* j, int32_t* k);

/* Device: writes table[3*i + {0,1,2}] = (class, j, k) for all i < M.
 * table: device int32, 3*M entries. Integer-exact. */
int lb_basis_table(lb_ctx* ctx, int N, int32_t* table);

/* ------------------------------------------------------------------ */
/* Nonzero structure constants (Eq. (11), Table 1 step 2.2)            */
/* ------------------------------------------------------------------ */

/* Number of ordered triples (m, n, s) with f_mns != 0 (which = 0) or
 * d_mns != 0 (which = 1). Runs the GPU count phase; synchronizes. */
int lb_fd_count(lb_ctx* ctx, int N, int which, int64_t* count);

/* Writes every ordered nonzero triple: mns[3*e + {0,1,2}] = (m, n, s) and
 * val[e] = f_mns or d_mns, grouped by m in increasing order. mns (device
 * int32, 3*cap) and val (device double, cap) must hold `cap` entries;
 * *count (host) receives the total. Fails with LB_ERR_INVALID_ARG when
 * cap < total (nothing is written then). Synchronizes. */
int lb_fd_enumerate(lb_ctx* ctx, int N, int which, int32_t* mns, double* val, int64_t cap, int64_t* count);

/* ------------------------------------------------------------------ */
/* Expansion and reconstruction (Eqs. (6), (7); Table 1 steps 2.1,     */
/* 2.6, 3.2)                                                           */
/* ------------------------------------------------------------------ */

/* a[b*M + j] = Re Tr(F_j A_b) for B Hermitian N x N complex matrices
 * A (device, B*N*N complex) -> a (device, B*M double). */
int lb_expand(lb_ctx* ctx, int N, int B, const double* A, double* a);

/* Coherence vectors of B pure states: V[b*M + j] = <psi_b| F_j |psi_b>.
 * psi: device, B*N complex (normalised by the caller). V: device, B*M. */
int lb_expand_pure(lb_ctx* ctx, int N, int B, const double* psi, double* V);

/* rho_b = 1/N + sum_j V[b*M + j] F_j (Eq. (7)); rho: device, B*N*N complex. */
int lb_reconstruct(lb_ctx* ctx, int N, int B, const double* V, double* rho);

/* ------------------------------------------------------------------ */
/* Dense data preparation (Eqs. (13)-(15); Table 1 steps 2.1-2.5)      */
/* ------------------------------------------------------------------ */

/* Builds Q = Q_H + Q_D (the paper's Q(t) + R) and K for a Hamiltonian H
 * (device, N*N complex, Hermitian) and a Kossakowski matrix gamma (device,
 * M*M complex, Hermitian, in the basis order above). Writes Q (device,
 * M rows of leading dimension ldq >= M doubles; columns M..ldq-1 are set to
 * zero) and K (device, M doubles). gamma is read assuming exact Hermiticity
 * (entries may be read from either triangle). The identity part of H is
 * irrelevant. FP64 throughout. */
int lindblad_prepare(lb_ctx* ctx, int N, const double* H, const double* gamma,
                     double* Q, int64_t ldq, double* K, unsigned flags);

/* ------------------------------------------------------------------ */
/* Sparse data preparation: gamma = sum_p g_p l_p l_p^dagger given by  */
/* jump operators (Sec. 2, spectral form of the Kossakowski matrix)    */
/* ------------------------------------------------------------------ */

/* An N x N complex matrix in CSR form; all arrays device memory. */
typedef struct lb_csr_c128 {
    const int64_t* rowptr; /* N+1 */
    const int64_t* col;    /* nnz */
    const double* val;     /* nnz complex (interleaved) */
    int64_t nnz;
} lb_csr_c128;

/* Phase 1 (count): the number of stored entries of Q for the Hamiltonian H
 * and P jump operators L_p with rates g_p >= 0 (rates: host, P doubles).
 * Each row s of Q holds the expansion of the adjoint generator applied to
 * F_s. A nonzero trace of L_p is moved into the Hamiltonian
 * (H += (i g_p / 2)(conj(c) L0 - c L0^dagger), c = Tr L_p / N, L0 = L_p - c).
 * Synchronizes; *nnz (host) receives the count. */
int lindblad_prepare_sparse_count(lb_ctx* ctx, int N, const lb_csr_c128* H, int P,
                                  const double* rates, const lb_csr_c128* L, int64_t* nnz);

/* Phase 2 (fill): writes Q in CSR form (rowptr: device int64 M+1; col:
 * device int64 nnz; val: device double nnz; columns sorted within a row)
 * and K (device, M doubles). nnz must be the value phase 1 returned. */
int lindblad_prepare_sparse_fill(lb_ctx* ctx, int N, const lb_csr_c128* H, int P,
                                 const double* rates, const lb_csr_c128* L, int64_t nnz,
                                 int64_t* rowptr, int64_t* col, double* val, double* K);

/* ------------------------------------------------------------------ */
/* RK4 propagation of dv/dt = Q v + K (Eq. (10); Table 1 step 3.1)      */
/* ------------------------------------------------------------------ */

/* Integrates B states over `steps` classic RK4 steps of size dt (weights
 * 1/6, 1/3, 1/3, 1/6; K constant). V (device, B*M doubles, state b at
 * V + b*M) holds v(0) on entry and v(steps*dt) on exit. Q: device, M rows
 * of leading dimension ldq. precision LB_FP64 uses Q directly; LB_FP32
 * requires Q32 (device float, same ldq) from lindblad_q_to_f32 and ignores
 * Q. Bit-for-bit deterministic for fixed inputs and launch configuration.
 * When Q (or Q32) starts on a 128-byte boundary and its rows are 128-byte
 * multiples (ldq a multiple of 16 in FP64, 32 in FP32), the stage GEMM stages
 * Q through LDS with full-line streaming loads; otherwise it loads the matrix
 * core operands directly. Both give identical results. */
int lindblad_propagate(lb_ctx* ctx, int64_t M, const double* Q, const float* Q32, int64_t ldq,
                       const double* K, double* V, int B, double dt, int64_t steps, int precision);

/* Allocation-free variant of lindblad_propagate, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). Same arguments, layout, ownership and
 * result (the same kernels and tile: bit for bit), but the integration's
 * buffers live in one static device array of LB_NOALLOC_SCRATCH_BYTES per GPU,
 * held from module load until the process ends; the call allocates no device
 * or pinned host memory and does not synchronize. Limit: the buffers must fit
 * the array -- 2 M doubles of packed states, stage vectors and split-K
 * partials (one state up to M = 699000; 16 states up to M of about 5000, i.e.
 * N = 70) -- else LB_ERR_UNSUPPORTED. Every call on a GPU uses that GPU's one array: calls
 * that overlap on one GPU (other streams or threads) race and must be
 * serialized by the caller. Other errors as lindblad_propagate. */
#define LB_NOALLOC_SCRATCH_BYTES (16u << 20)
int lindblad_propagate_noalloc(lb_ctx* ctx, int64_t M, const double* Q, const float* Q32, int64_t ldq,
                               const double* K, double* V, int B, double dt, int64_t steps, int precision);

/* Q32[i*ldq + j] = (float)Q[i*ldq + j] for i < M, j < ldq (device buffers). */
int lindblad_q_to_f32(lb_ctx* ctx, int64_t M, const double* Q, int64_t ldq, float* Q32);

/* CSR variant: Q given by rowptr/col/val (device, as written by
 * lindblad_prepare_sparse_fill). FP64. */
int lindblad_propagate_csr(lb_ctx* ctx, int64_t M, const int64_t* rowptr, const int64_t* col,
                           const double* val, const double* K, double* V, int B,
                           double dt, int64_t steps);

/* Periodically rocked dimer (Sec. 3, Eq. (16)): H(t) = H0 + eps(t) H1 with
 * the square wave eps(t) = E + A Theta(t), Theta = +1 on [0, T/2) and -1 on
 * [T/2, T), period T. Q_H is linear in H and the drive adds nothing to K, so
 * the system is dv/dt = (Q0 + eps(t) Q1) v + K with Q0 (from H0 and the jump
 * operators) and Q1 (from H1 alone, no jump operators) as written by
 * lindblad_prepare_sparse_fill, and K that of Q0. Classic RK4 over steps k0,
 * k0 + 1, ..., k0 + steps - 1 of the time grid t0 + k dt: step k evaluates eps
 * at t0 + k dt and t0 + (k + 1/2) dt from the right and at t0 + (k + 1) dt as
 * the limit from the left, i.e. each step sees the drive of
 * the interval it integrates, so steps that end on a switch (T/2 a multiple of
 * dt, as with 20000 steps per period) integrate one constant system and the
 * scheme keeps fourth order. A run split at step k0 and continued with the
 * same t0 and the step offset k0 is bit-identical to the uninterrupted run
 * (every stage time is formed from t0 and the global step index). FP64, B
 * states in V (B*M), in place; errors as lindblad_propagate_csr, plus
 * LB_ERR_INVALID_ARG for a non-finite t0, E, A, T <= 0 or k0 < 0, and (when
 * steps > 0) unless every switch lies on the step grid: T/(2 dt) and t0/dt
 * must be integers within a relative 1e-9, so no step straddles a switch and
 * the result does not depend on how a stage at a switch would be evaluated. */
int lindblad_propagate_csr_drive(lb_ctx* ctx, int64_t M, const int64_t* rowptr0, const int64_t* col0,
                                 const double* val0, const int64_t* rowptr1, const int64_t* col1,
                                 const double* val1, const double* K, double* V, int B, double dt,
                                 int64_t steps, double t0, int64_t k0, double E, double A, double T);

/* Batched variant: R independent systems of the same M (e.g. ensemble
 * realizations), Q[r], K[r], V[r] device pointers given in host arrays of
 * length R; each V[r] holds B states. One launch per RK4 stage covers all
 * systems. Same precision rules as lindblad_propagate (Q32 may be NULL for
 * LB_FP64). */
int lindblad_propagate_batched(lb_ctx* ctx, int R, int64_t M, const double* const* Q,
                               const float* const* Q32, int64_t ldq, const double* const* K,
                               double* const* V, int B, double dt, int64_t steps, int precision);

/* Records the RK4 stage launches of `steps` steps into a HIP graph on first
 * use for a given (M, B, ldq, precision, buffers, dt, steps) and replays it
 * afterwards; otherwise identical to lindblad_propagate. A captured graph
 * keeps the raw Q, K and V pointers and its own device buffers; a context
 * keeps at most 8 graphs and frees the least recently used one (after
 * synchronizing its stream) when a ninth is captured. */
int lindblad_propagate_graph(lb_ctx* ctx, int64_t M, const double* Q, const float* Q32, int64_t ldq,
                             const double* K, double* V, int B, double dt, int64_t steps, int precision);

/* Frees every graph the context has captured (after synchronizing its stream)
 * and their buffers; *freed (may be NULL) receives how many. Call it before
 * freeing the Q, K or V buffers of captured graphs. */
int lindblad_graph_clear(lb_ctx* ctx, int* freed);

/* ------------------------------------------------------------------ */
/* Saved systems (Sec. 5: the integration runs from prepared, stored data) */
/* ------------------------------------------------------------------ */

#define LB_SYSTEM_DENSE 0
#define LB_SYSTEM_CSR 1

/* A prepared system in device memory: dense Q and K as written by
 * lindblad_prepare, or CSR Q and K as written by lindblad_prepare_sparse_fill. */
typedef struct lb_system {
    int kind;          /* LB_SYSTEM_DENSE or LB_SYSTEM_CSR */
    int N;             /* Hilbert-space dimension, M = N*N - 1 */
    int64_t ldq;       /* dense: leading dimension of Q (>= M) */
    int64_t nnz;       /* CSR: stored entries */
    double* Q;         /* dense: M x ldq, row-major */
    int64_t* rowptr;   /* CSR: M + 1 */
    int64_t* col;      /* CSR: nnz */
    double* val;       /* CSR: nnz */
    double* K;         /* M */
} lb_system;

/* Writes the system to a file: an 80-byte header (magic "LBSYSTEM", version,
 * kind, N, M, nnz, a hash of the payload computed on the device), then Q (dense:
 * M rows of M doubles, whatever ldq; CSR: rowptr, col, val) and K, in the
 * host's (little-endian) byte order. Streams through pinned staging buffers;
 * returns after the file is written and flushed. Errors: LB_ERR_INVALID_ARG
 * (sizes, null pointers, CSR rowptr[M] != nnz), LB_ERR_IO, LB_ERR_OOM,
 * LB_ERR_DEVICE. */
int lindblad_save_system(lb_ctx* ctx, const char* path, const lb_system* sys);

/* Reads only the header (host, no device work): fills kind, N and nnz of
 * *sys, so that the caller can allocate the buffers; leaves the rest. */
int lindblad_load_system_info(const char* path, lb_system* sys);

/* Loads a saved system into caller-allocated device buffers described by *sys
 * (kind, N, nnz must match the file; dense Q may have any ldq >= M, its padding
 * columns are zeroed). The payload hash is recomputed on the device and
 * compared: LB_ERR_IO if the file is not a valid saved system or is corrupt,
 * LB_ERR_INVALID_ARG if the buffers describe another system. Synchronous. */
int lindblad_load_system(lb_ctx* ctx, const char* path, lb_system* sys);

/* ------------------------------------------------------------------ */
/* Steady state (Sec. 3: the asymptotic state rho_inf, L(rho_inf) = 0) */
/* ------------------------------------------------------------------ */

/* Eigen-decomposition of a Hermitian matrix, A = Z diag(w) Z^H: the energy
 * eigenbasis of H in which the steady-state preconditioner is diagonal. A is
 * N x N complex (interleaved re, im), column-major with lda >= N, on the
 * device, Hermitian on entry and overwritten (its diagonal ends as w); w
 * receives N doubles (not sorted), Z the N x N eigenvectors (column-major,
 * ldz >= N). Cyclic two-sided Jacobi in FP64 until the off-diagonal norm is
 * below 1e-14 ||A||_F; *sweeps (may be NULL) receives the number of sweeps.
 * Errors: LB_ERR_INVALID_ARG, LB_ERR_NO_CONVERGENCE (40 sweeps). */
int lb_eigh(lb_ctx* ctx, int N, double* A, int lda, double* w, double* Z, int ldz, int* sweeps);

/* Steady-state preconditioner for a Lindbladian given by H and jump operators
 * L_p with rates g_p (the form of lindblad_prepare_sparse): the secular
 * approximation of L in the energy eigenbasis of H, inverted exactly. There,
 * each coherence X_ab (a != b) decays at -i(E_a - E_b) - (G_aa + G_bb)/2 +
 * sum_p g_p L_p,aa conj(L_p,bb) with G = sum_p g_p L_p^H L_p, and the
 * populations follow the rate equations with rates W_ab = sum_p g_p |L_p,ab|^2.
 * It keeps GMRES iteration counts low where H's frequencies dwarf the
 * dissipation (the dimer). Set-up: H and every L_p densified, H diagonalised
 * (lb_eigh), two complex N x N GEMMs per jump operator, Gauss-Jordan inversion
 * of the (N+1) x (N+1) bordered rate matrix; holds about 4 N^2 complex and
 * (N+1)^2 real numbers of device memory until lindblad_secular_destroy. Each
 * application costs four complex N x N GEMMs. H and L as for
 * lindblad_prepare_sparse_count (device CSR, rates on the host). Errors:
 * LB_ERR_INVALID_ARG (sizes, null pointers, a singular rate matrix),
 * LB_ERR_OOM, LB_ERR_NO_CONVERGENCE (eigensolver), LB_ERR_DEVICE. */
typedef struct lb_secular lb_secular;
int lindblad_secular_create(lb_ctx* ctx, int N, const lb_csr_c128* H, int P, const double* rates,
                            const lb_csr_c128* L, lb_secular** out);
int lindblad_secular_destroy(lb_secular* pre);

/* Outcome of an iterative solve. */
typedef struct lb_solve_info {
    int64_t iterations; /* Krylov iterations (one operator application each) over all cycles */
    int64_t restarts;   /* cycles after the first */
    double residual;    /* ||Q v + K||_2 / ||K||_2 of the returned v, recomputed from v */
    int converged;      /* 1 if residual <= tol */
} lb_solve_info;

/* The stationary point of Eq. (10): v with Q v = -K, the coherence vector
 * (Eq. (7)) of rho_inf. Dense Q (M rows, leading dimension ldq >= M) and K as
 * written by lindblad_prepare; v (M doubles, device) receives the solution.
 * FP64 restarted GMRES from v = 0 with classical Gram-Schmidt applied twice;
 * the Krylov basis (restart + 1 vectors of M doubles) is allocated for the
 * call and freed before it returns. Stops when ||Q v + K||_2 <= tol ||K||_2
 * (K = 0 gives v = 0 at once) or after maxit iterations, restarting every
 * `restart` iterations (1 <= restart <= 8192). Errors: LB_ERR_INVALID_ARG
 * (null pointers, sizes, tol not in (0, 1), maxit < 1), LB_ERR_OOM (basis does
 * not fit), LB_ERR_NO_CONVERGENCE (v holds the last iterate, *info filled).
 * pre (may be NULL) is a preconditioner for the same system (M = N^2 - 1),
 * applied on the right. info may be NULL. Results are deterministic
 * (fixed-order reductions). */
int lindblad_steady_state(lb_ctx* ctx, int64_t M, const double* Q, int64_t ldq, const double* K,
                          const lb_secular* pre, double* v, double tol, int64_t maxit,
                          int64_t restart, lb_solve_info* info);

/* The same for Q in CSR form (as written by lindblad_prepare_sparse_fill). */
int lindblad_steady_state_csr(lb_ctx* ctx, int64_t M, const int64_t* rowptr, const int64_t* col,
                              const double* val, const double* K, const lb_secular* pre, double* v,
                              double tol, int64_t maxit, int64_t restart, lb_solve_info* info);

/* ------------------------------------------------------------------ */
/* Spectrum of the generator (Sec. 5, Fig. 5)                         */
/* ------------------------------------------------------------------ */

/* Largest M accepted by lindblad_spectrum and lb_hessenberg: M^2 < 2^31 (the
 * one-workgroup solver addresses blocks with 32-bit offsets). N = 200 gives
 * M = 39999. */
#define LB_SPECTRUM_MAX_M 46340

/* Reduces the real M x M matrix A (row-major, lda >= M, device) in place to
 * upper Hessenberg form by an orthogonal similarity (Householder reflectors
 * applied from both sides, one column at a time): entries below the
 * subdiagonal are set to exactly zero, the eigenvalues are kept. The first
 * stage of lindblad_spectrum, exported for tests. Errors: LB_ERR_INVALID_ARG
 * (M < 1, M > LB_SPECTRUM_MAX_M, lda < M, null A), LB_ERR_OOM, LB_ERR_DEVICE.
 * Asynchronous on the context stream. */
int lb_hessenberg(lb_ctx* ctx, int64_t M, double* A, int64_t lda);

typedef struct lb_spectrum_info {
    int64_t sweeps;        /* QR sweeps over all blocks */
    int64_t chain_steps;   /* chain steps over all sweeps */
    int64_t updates;       /* 2- or 3-entry row and column pieces the reflectors update
                              (10 flops each): b (na^2 + 3 na - 7) per b-bulge sweep
                              over an na-row block */
    int64_t rounds;        /* windowed rounds of the sweeps over blocks above 256 rows */
    int64_t product_flops; /* flops of those rounds' matrix products outside the windows:
                              2 w^2 per row or column of the block a w-row window
                              updates (the dense count; the band of the window
                              factor lets the kernels skip about 30 % of it) */
} lb_spectrum_info;

/* Eigenvalues of the real generator Q of the ODE dv/dt = Qv + K (Eq. (10);
 * M x M, row-major, ldq >= M, device, not modified). With rho = 1/N + sum
 * v_n F_n (Eq. (7)) the Lindbladian acts on the coordinates (1, v) as
 * [[0, 0], [K, Q]], so its spectrum is 0 and these M = N^2 - 1 values, the
 * ones Fig. 5 histograms. lam receives M complex values (interleaved re, im:
 * 2M doubles, device): complex-conjugate pairs adjacent with the positive
 * imaginary part first, otherwise in no particular order. Works on a copy of Q
 * in the context's workspace (M^2 doubles): Householder reduction to Hessenberg
 * form, then Francis' implicit double-shift QR iteration (eigenvalues only)
 * whose shifts are the eigenvalues of the trailing block: sweeps over blocks
 * above 256 rows move up to 64 bulges as chains of 8, each chased inside a
 * 96 x 96 window with the rest of the block updated by matrix products, and
 * blocks of at most 256 rows are finished by one workgroup (up to 16 bulges
 * per sweep); a block splits off where a subdiagonal entry falls below
 * eps (|h_k-1,k-1| + |h_kk|), or below eps ||Q||_F once ten sweeps have passed
 * without a split and below sqrt(M) eps ||Q||_F after twenty (clusters at the
 * rounding floor). *info (may be NULL) receives the iteration
 * counts. Synchronous. Errors: LB_ERR_INVALID_ARG (M < 1, M >
 * LB_SPECTRUM_MAX_M, ldq < M, null pointers), LB_ERR_OOM,
 * LB_ERR_NO_CONVERGENCE (120 sweeps without a split; lam is then not valid),
 * LB_ERR_DEVICE. */
int lindblad_spectrum(lb_ctx* ctx, int64_t M, const double* Q, int64_t ldq, double* lam, lb_spectrum_info* info);

/* Counts of the n complex values lam (interleaved re, im, device) per cell of
 * the nx x ny grid over [re0, re1) x [im0, im1) (Fig. 5: a 100 x 100 grid, each
 * count divided by the cell area). A value lands in column
 * floor((re - re0) / dx), dx = (re1 - re0) / nx, and row floor((im - im0) / dy),
 * dy = (im1 - im0) / ny, and is counted when 0 <= (re - re0) / dx < nx and
 * 0 <= (im - im0) / dy < ny; others (NaN included) are not. counts: ny x nx
 * int64, row-major (row = imaginary cell), device, overwritten. Errors:
 * LB_ERR_INVALID_ARG (n < 0, nx or ny < 1, nx * ny > 2^26, re1 <= re0,
 * im1 <= im0, non-finite bounds, null pointers), LB_ERR_DEVICE. Asynchronous. */
int lindblad_spectrum_histogram(lb_ctx* ctx, int64_t n, const double* lam, double re0, double re1, double im0,
                                double im1, int nx, int ny, int64_t* counts);

/* ------------------------------------------------------------------ */
/* Measurement                                                        */
/* ------------------------------------------------------------------ */

/* Dense FP64 products on the matrix cores, the building block of the
 * preconditioner's basis changes and the blocked Hessenberg reduction; exported
 * for tests. All matrices are column-major device arrays with leading
 * dimensions (elements), asynchronous on the context stream, no allocation.
 * lb_gemm_f64: C = alpha op(A) op(B) + beta C, C m x n, op(A) m x k, op(B) k x n;
 * op is the transpose when trans_a / trans_b is nonzero (then A is stored k x m,
 * B n x k). With beta = 0, C is not read.
 * lb_gemm_c128: C = op(A) op(B) on complex128 (interleaved re, im; leading
 * dimensions in complex elements); op is the conjugate transpose when conj_a /
 * conj_b is nonzero. work (may be NULL) is caller-owned device scratch of
 * work_elems complex values: when the grid of 64 x 64 tiles of C is small, k
 * is split into up to 8 slices whose dense m x n partial products go there and
 * are then summed in slice order (as many slices as the scratch holds; none
 * without it). The result depends on the slicing only through rounding.
 * Errors: LB_ERR_INVALID_ARG (negative sizes, leading dimension below the
 * stored rows, null operands with nonzero sizes, work_elems < 0 or a NULL
 * work with work_elems > 0). */
int lb_gemm_f64(lb_ctx* ctx, int trans_a, int trans_b, int64_t m, int64_t n, int64_t k, double alpha,
                const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc);
int lb_gemm_c128(lb_ctx* ctx, int conj_a, int conj_b, int64_t m, int64_t n, int64_t k, const double* A,
                 int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc, double* work,
                 int64_t work_elems);

/* Read-stream bandwidth of the context's device in GB/s (1e9 bytes/s): a
 * reduction over a buffer of `bytes` (allocated and freed by the call) with
 * 16-byte nontemporal loads, timed with HIP events, the best of five grid
 * sizes. The practical ceiling next to the published HBM peak for the
 * bandwidth-bound kernels. Synchronous. */
int lb_read_bandwidth(lb_ctx* ctx, size_t bytes, double* gbs);

/* ------------------------------------------------------------------ */
/* Tuning                                                             */
/* ------------------------------------------------------------------ */

/* Times the candidate GEMM tile shapes for (M, B, precision) on the context
 * stream and keeps the fastest for later propagate calls in this process
 * (and in the cache file named by the LB_TUNE_CACHE environment variable,
 * if set). Q/Q32 and K as for lindblad_propagate; V is scratch (B*M). */
int lindblad_autotune(lb_ctx* ctx, int64_t M, const double* Q, const float* Q32, int64_t ldq,
                      const double* K, double* V, int B, int precision);

/* Measurement: average duration in milliseconds of the dominant RK4 stage
 * kernel (the stage GEMM, or the stage GEMV for one FP64 state) for R
 * systems, over `iters` back-to-back launches timed with HIP events on the
 * context stream. Arguments as for lindblad_propagate_batched; the states are
 * read but not advanced. Synchronizes. */
int lindblad_time_stage(lb_ctx* ctx, int R, int64_t M, const double* const* Q, const float* const* Q32,
                        int64_t ldq, const double* const* K, double* const* V, int B, int precision,
                        int iters, double* avg_ms);

/* Sets the tile shape propagate uses for (M, B, precision) in this context:
 * rows per wave (16..128, multiple of 16; combinations without a compiled
 * kernel are rejected at propagate time), k-slab length (multiple of 16) and
 * waves per workgroup (1..4). */
int lindblad_set_tile(lb_ctx* ctx, int64_t M, int B, int precision, int rows, int kslab, int waves);

/* Describes the tile shape propagate will use for (M, B, precision):
 * rows per wave, k-slab length, waves per workgroup, and whether it came
 * from the tuner (1) or the default table (0). Host only. */
int lindblad_tile_info(lb_ctx* ctx, int64_t M, int B, int precision, int* rows, int* kslab,
                       int* waves, int* tuned);

/* ------------------------------------------------------------------ */
/* Serving: continuous batching of prepare + propagate requests         */
/* ------------------------------------------------------------------ */

#define LB_REQ_DENSE 0
#define LB_REQ_SPARSE 1
#define LB_REQ_SYSTEM 2
#define LB_REQ_MAX_JUMPS 8
#define LB_SYSTEM_BATCH 16            /* states integrated together on one registered system */

/* One request: prepare the ODE system of a Lindbladian of dimension N and
 * integrate B states for `steps` RK4 steps (kinds LB_REQ_DENSE, LB_REQ_SPARSE),
 * or integrate B <= LB_SYSTEM_BATCH states on a system registered with
 * lindblad_server_register (kind LB_REQ_SYSTEM: only system, V0, Vout, B, dt,
 * steps and precision are read). All pointers are device memory owned by the
 * caller and must stay valid until the request completes. */
typedef struct lb_request {
    int kind;                         /* LB_REQ_DENSE or LB_REQ_SPARSE */
    int N;
    const double* H;                  /* dense: N*N complex Hamiltonian */
    const double* gamma;              /* dense: M*M complex Kossakowski matrix */
    lb_csr_c128 Hs;                   /* sparse: Hamiltonian (CSR) */
    int P;                            /* sparse: number of jump operators */
    double rates[LB_REQ_MAX_JUMPS];   /* sparse: rates g_p */
    lb_csr_c128 L[LB_REQ_MAX_JUMPS];  /* sparse: jump operators (CSR) */
    const double* V0;                 /* B*M initial coherence vectors */
    double* Vout;                     /* B*M results v(steps*dt) */
    int B;
    double dt;
    int64_t steps;
    int precision;                    /* dense: LB_FP64 or LB_FP32; sparse: LB_FP64 */
    int64_t system;                   /* LB_REQ_SYSTEM: id from lindblad_server_register */
} lb_request;

typedef struct lb_server lb_server;

/* Starts a server on `device` with `max_slots` worker slots (each a thread with
 * its own stream and context, workspace pre-sized for N <= max_N), an HBM
 * budget for the per-request buffers (Q/CSR, K, state blocks), and batches of
 * up to `max_batch` requests: queued requests with the same inputs (the same
 * H and gamma, or CSR, arrays, the same dt, steps and precision) share one
 * preparation and one pass (their states packed into a block of at most
 * LB_SYSTEM_BATCH), and dense requests of the same N, dt, steps and precision
 * on other inputs are integrated in the same launches. Admission keeps
 * submission order: the oldest waiting request starts as soon as a slot is
 * free and its footprint fits in the budget. With max_batch = 1 every request
 * runs alone. A request's result is the same bit for bit alone and batched. */
int lindblad_server_create(int device, size_t hbm_budget_bytes, int max_slots, int max_batch, int max_N,
                           lb_server** srv);
/* Queues a request (thread-safe; copies the descriptor, not the data).
 * LB_ERR_ADMISSION if its footprint cannot fit in the budget next to the
 * registered systems. A queued request that a later registration has left
 * without room is failed with LB_ERR_ADMISSION (lindblad_server_wait
 * returns it) instead of blocking the requests behind it. */
int lindblad_server_submit(lb_server* srv, const lb_request* req, int64_t* ticket);
/* Resident systems: many initial states integrated on the same Lindbladian
 * (an ensemble of initial conditions). Prepares Q and K of the Lindbladian in
 * `req` (kind LB_REQ_DENSE with H, gamma, precision; or LB_REQ_SPARSE with
 * Hs, P, rates, L) once, synchronously, and keeps them in device memory
 * (counted against the budget) until released. Queued LB_REQ_SYSTEM requests
 * on the same system with the same dt, steps and precision are integrated
 * together, up to LB_SYSTEM_BATCH states per pass over Q; each state's result
 * is the same bit for bit whichever requests share its pass (dense systems
 * always run the 16-state matrix-core path, sparse ones the CSR kernel, whose
 * per-state arithmetic does not depend on the other states).
 * LB_ERR_ADMISSION when the system cannot fit in the budget next to the
 * systems already registered and the largest queued request (it waits while
 * running requests hold memory). */
int lindblad_server_register(lb_server* srv, const lb_request* req, int64_t* system);
/* Releases a registered system; its memory is freed once no queued or
 * running request uses it. Further requests on it fail with LB_ERR_INVALID_ARG. */
int lindblad_server_release(lb_server* srv, int64_t system);
/* *done = 1 once the request has finished (successfully or not). */
int lindblad_server_poll(lb_server* srv, int64_t ticket, int* done);
/* Blocks until the request has finished; returns its status. */
int lindblad_server_wait(lb_server* srv, int64_t ticket);
/* Submission, start and completion times of a request (seconds, steady clock). */
int lindblad_server_times(lb_server* srv, int64_t ticket, double* t_submit, double* t_start, double* t_end);
/* Completed requests, peak budget use (bytes), batches run, requests that ran in batches of > 1. */
int lindblad_server_stats(lb_server* srv, int64_t* completed, size_t* peak_bytes, int64_t* batches,
                          int64_t* batched_requests);
/* Cancels the requests still queued (their status becomes LB_ERR_CANCELLED),
 * waits for the running ones, frees the registered systems and releases the
 * server. No other call on the server may run concurrently with it, and its
 * tickets are invalid afterwards. */
int lindblad_server_destroy(lb_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* LINDBLAD_H */
