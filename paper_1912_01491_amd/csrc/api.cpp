// C ABI: context management, argument validation and dispatch to the kernels.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <chrono>

#include "lb_internal.h"

static thread_local char g_err[512] = "";

void lb_set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int lb_fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int lb_use_device(lb_ctx* c) {
    LB_HIP(hipSetDevice(c->device));
    return LB_OK;
}

int lb_ws_reserve(lb_ctx* c, size_t bytes) {
    if (bytes <= c->ws_bytes) return LB_OK;
    // the old buffer may still be in use by enqueued work
    LB_HIP(hipStreamSynchronize(c->stream));
    if (c->ws) {
        LB_HIP(hipFree(c->ws));
        c->ws = nullptr;
        c->ws_bytes = 0;
    }
    size_t want = lb_align(bytes + bytes / 8, 1 << 20);
    hipError_t e = hipMalloc(&c->ws, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c->ws = nullptr;
        return lb_fail(LB_ERR_OOM, "workspace allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
    }
    c->ws_bytes = want;
    return LB_OK;
}

int lb_host_reserve(lb_ctx* c, size_t bytes) {
    if (bytes <= c->host_bytes) return LB_OK;
    LB_HIP(hipStreamSynchronize(c->stream));
    if (c->host) {
        LB_HIP(hipHostFree(c->host));
        c->host = nullptr;
        c->host_bytes = 0;
    }
    size_t want = lb_align(bytes, 1 << 16);
    hipError_t e = hipHostMalloc(&c->host, want, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c->host = nullptr;
        return lb_fail(LB_ERR_OOM, "pinned host allocation of %zu bytes failed", want);
    }
    c->host_bytes = want;
    return LB_OK;
}

#define CHECK_CTX(c)                                                   \
    do {                                                               \
        if (!(c)) return lb_fail(LB_ERR_INVALID_ARG, "null context"); \
        int _rc = lb_use_device(c);                                    \
        if (_rc) return _rc;                                           \
    } while (0)

#define CHECK_N(N)                                                                               \
    do {                                                                                         \
        if ((N) < 2 || (N) > LB_MAX_N) return lb_fail(LB_ERR_INVALID_ARG, "N=%d out of range [2, %d]", (N), LB_MAX_N); \
    } while (0)

#define CHECK_PTR(p)                                                        \
    do {                                                                    \
        if (!(p)) return lb_fail(LB_ERR_INVALID_ARG, "null pointer: %s", #p); \
    } while (0)

void lb_report(lb_ctx* c, const char* stage, double fraction) {
    static thread_local std::chrono::steady_clock::time_point last;
    static thread_local const char* last_stage = nullptr;
    if (!c->progress) return;
    const auto now = std::chrono::steady_clock::now();
    if (fraction < 1.0 && stage == last_stage && now - last < std::chrono::seconds(2)) return;
    last = now;
    last_stage = stage;
    c->progress(stage, fraction, c->progress_user);
}

extern "C" {

int lb_version(void) { return 100; }

const char* lb_last_error(void) { return g_err; }

int lb_create(lb_ctx** out, int device, void* stream) {
    if (!out) return lb_fail(LB_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    int n = 0;
    LB_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return lb_fail(LB_ERR_INVALID_ARG, "device %d not present (%d devices)", device, n);
    LB_HIP(hipSetDevice(device));
    const int rc = lb_scratch_init(device);  // the allocation-free propagate's static array, once per device
    if (rc) return rc;
    lb_ctx* c = new lb_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;  // NULL: the device's default stream
    *out = c;
    return LB_OK;
}

int lb_destroy(lb_ctx* c) {
    if (!c) return LB_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->graphs) lb_graph_free(kv.second);
    if (c->aux) {
        (void)hipStreamSynchronize(c->aux);
        (void)hipStreamDestroy(c->aux);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->ws) (void)hipFree(c->ws);
    if (c->host) (void)hipHostFree(c->host);
    delete c;
    return LB_OK;
}

int lb_set_stream(lb_ctx* c, void* stream) {
    CHECK_CTX(c);
    LB_HIP(hipStreamSynchronize(c->stream));
    c->stream = (hipStream_t)stream;
    return LB_OK;
}

int lb_set_progress(lb_ctx* c, lb_progress_fn fn, void* user) {
    CHECK_CTX(c);
    c->progress = fn;
    c->progress_user = user;
    return LB_OK;
}

int lb_sync(lb_ctx* c) {
    CHECK_CTX(c);
    LB_HIP(hipStreamSynchronize(c->stream));
    return LB_OK;
}

int lb_basis_index(int N, int64_t i, int32_t* cls, int32_t* j, int32_t* k) {
    CHECK_N(N);
    CHECK_PTR(cls);
    CHECK_PTR(j);
    CHECK_PTR(k);
    const int64_t M = (int64_t)N * N - 1;
    if (i < 0 || i >= M) return lb_fail(LB_ERR_INVALID_ARG, "index %lld out of range [0, %lld)", (long long)i, (long long)M);
    int c_, j_, k_;
    lb_decode(N, i, c_, j_, k_);
    *cls = c_;
    *j = j_;
    *k = k_;
    return LB_OK;
}

int lb_basis_table(lb_ctx* c, int N, int32_t* table) {
    CHECK_CTX(c);
    CHECK_N(N);
    CHECK_PTR(table);
    return lb_impl_basis_table(c, N, table);
}

int lb_fd_count(lb_ctx* c, int N, int which, int64_t* count) {
    CHECK_CTX(c);
    CHECK_N(N);
    CHECK_PTR(count);
    if (which != 0 && which != 1) return lb_fail(LB_ERR_INVALID_ARG, "which must be 0 (f) or 1 (d)");
    return lb_impl_fd_count(c, N, which, count, nullptr);
}

int lb_fd_enumerate(lb_ctx* c, int N, int which, int32_t* mns, double* val, int64_t cap, int64_t* count) {
    CHECK_CTX(c);
    CHECK_N(N);
    CHECK_PTR(count);
    if (which != 0 && which != 1) return lb_fail(LB_ERR_INVALID_ARG, "which must be 0 (f) or 1 (d)");
    int64_t total = 0;
    int rc = lb_impl_fd_count(c, N, which, &total, nullptr);
    if (rc) return rc;
    *count = total;
    if (cap < total) return lb_fail(LB_ERR_INVALID_ARG, "capacity %lld < %lld nonzeros", (long long)cap, (long long)total);
    if (total == 0) return LB_OK;
    CHECK_PTR(mns);
    CHECK_PTR(val);
    const int64_t M = (int64_t)N * N - 1;
    const int64_t* offsets = (const int64_t*)c->ws + M;
    rc = lb_impl_fd_fill(c, N, which, offsets, mns, val);
    if (rc) return rc;
    LB_HIP(hipStreamSynchronize(c->stream));
    return LB_OK;
}

int lb_expand(lb_ctx* c, int N, int B, const double* A, double* a) {
    CHECK_CTX(c);
    CHECK_N(N);
    CHECK_PTR(A);
    CHECK_PTR(a);
    if (B < 1) return lb_fail(LB_ERR_INVALID_ARG, "B=%d < 1", B);
    return lb_impl_expand(c, N, B, A, a, 1.0);
}

int lb_expand_pure(lb_ctx* c, int N, int B, const double* psi, double* V) {
    CHECK_CTX(c);
    CHECK_N(N);
    CHECK_PTR(psi);
    CHECK_PTR(V);
    if (B < 1) return lb_fail(LB_ERR_INVALID_ARG, "B=%d < 1", B);
    return lb_impl_expand_pure(c, N, B, psi, V);
}

int lb_reconstruct(lb_ctx* c, int N, int B, const double* V, double* rho) {
    CHECK_CTX(c);
    CHECK_N(N);
    CHECK_PTR(V);
    CHECK_PTR(rho);
    if (B < 1) return lb_fail(LB_ERR_INVALID_ARG, "B=%d < 1", B);
    return lb_impl_reconstruct(c, N, B, V, rho);
}

int lindblad_prepare(lb_ctx* c, int N, const double* H, const double* gamma, double* Q, int64_t ldq, double* K,
                     unsigned flags) {
    CHECK_CTX(c);
    CHECK_N(N);
    CHECK_PTR(H);
    CHECK_PTR(gamma);
    CHECK_PTR(Q);
    CHECK_PTR(K);
    const int64_t M = (int64_t)N * N - 1;
    if (ldq < M) return lb_fail(LB_ERR_INVALID_ARG, "ldq=%lld < M=%lld", (long long)ldq, (long long)M);
    if (((uintptr_t)gamma) % 16 || ((uintptr_t)H) % 16)
        return lb_fail(LB_ERR_INVALID_ARG, "H and gamma must be 16-byte aligned complex arrays");
    if (flags & LB_CHECK_HERMITIAN) {
        double dev = 0, mx = 0;
        int rc = lb_impl_hermitian_check(c, N, H, &dev, &mx);
        if (rc) return rc;
        if (dev > 1e-12 * (mx > 1 ? mx : 1)) return lb_fail(LB_ERR_NOT_HERMITIAN, "H is not Hermitian (max dev %g)", dev);
        rc = lb_impl_hermitian_check(c, M, gamma, &dev, &mx);
        if (rc) return rc;
        if (dev > 1e-12 * (mx > 1 ? mx : 1))
            return lb_fail(LB_ERR_NOT_HERMITIAN, "gamma is not Hermitian (max dev %g)", dev);
    }
    return lb_impl_prepare_dense(c, N, H, gamma, Q, ldq, K);
}

int lindblad_prepare_sparse_count(lb_ctx* c, int N, const lb_csr_c128* H, int P, const double* rates,
                                  const lb_csr_c128* L, int64_t* nnz) {
    CHECK_CTX(c);
    CHECK_N(N);
    CHECK_PTR(H);
    CHECK_PTR(nnz);
    if (P < 0 || (P > 0 && (!rates || !L))) return lb_fail(LB_ERR_INVALID_ARG, "bad jump-operator arguments");
    for (int p = 0; p < P; ++p)
        if (!(rates[p] >= 0) || !isfinite(rates[p])) return lb_fail(LB_ERR_INVALID_ARG, "rate %d must be finite and >= 0", p);
    return lb_impl_sparse(c, N, H, P, rates, L, nnz, nullptr, nullptr, nullptr, nullptr);
}

int lindblad_prepare_sparse_fill(lb_ctx* c, int N, const lb_csr_c128* H, int P, const double* rates,
                                 const lb_csr_c128* L, int64_t nnz, int64_t* rowptr, int64_t* col, double* val,
                                 double* K) {
    CHECK_CTX(c);
    CHECK_N(N);
    CHECK_PTR(H);
    CHECK_PTR(rowptr);
    CHECK_PTR(K);
    if (nnz > 0) {
        CHECK_PTR(col);
        CHECK_PTR(val);
    }
    if (P < 0 || (P > 0 && (!rates || !L))) return lb_fail(LB_ERR_INVALID_ARG, "bad jump-operator arguments");
    for (int p = 0; p < P; ++p)
        if (!(rates[p] >= 0) || !isfinite(rates[p])) return lb_fail(LB_ERR_INVALID_ARG, "rate %d must be finite and >= 0", p);
    int64_t n = nnz;
    return lb_impl_sparse(c, N, H, P, rates, L, &n, rowptr, col, val, K);
}

static int check_prop(int64_t M, int64_t ldq, int B, double dt, int64_t steps, int precision) {
    if (M < 3 || M > (int64_t)LB_MAX_N * LB_MAX_N - 1) return lb_fail(LB_ERR_INVALID_ARG, "M=%lld out of range", (long long)M);
    if (ldq < M) return lb_fail(LB_ERR_INVALID_ARG, "ldq < M");
    if (B < 1 || B > 64) return lb_fail(LB_ERR_INVALID_ARG, "B=%d out of range [1, 64]", B);
    if (!isfinite(dt)) return lb_fail(LB_ERR_INVALID_ARG, "dt is not finite");
    if (steps < 0) return lb_fail(LB_ERR_INVALID_ARG, "steps < 0");
    if (precision != LB_FP64 && precision != LB_FP32) return lb_fail(LB_ERR_INVALID_ARG, "unknown precision %d", precision);
    return LB_OK;
}

int lindblad_propagate(lb_ctx* c, int64_t M, const double* Q, const float* Q32, int64_t ldq, const double* K,
                       double* V, int B, double dt, int64_t steps, int precision) {
    CHECK_CTX(c);
    int rc = check_prop(M, ldq, B, dt, steps, precision);
    if (rc) return rc;
    CHECK_PTR(K);
    CHECK_PTR(V);
    if (precision == LB_FP64) CHECK_PTR(Q);
    else CHECK_PTR(Q32);
    lb_prop_sys s{Q, Q32, K, V};
    return lb_impl_propagate(c, 1, M, &s, ldq, B, dt, steps, precision, nullptr);
}

int lindblad_propagate_noalloc(lb_ctx* c, int64_t M, const double* Q, const float* Q32, int64_t ldq,
                               const double* K, double* V, int B, double dt, int64_t steps, int precision) {
    CHECK_CTX(c);
    int rc = check_prop(M, ldq, B, dt, steps, precision);
    if (rc) return rc;
    CHECK_PTR(K);
    CHECK_PTR(V);
    if (precision == LB_FP64) CHECK_PTR(Q);
    else CHECK_PTR(Q32);
    lb_prop_sys s{Q, Q32, K, V};
    return lb_impl_propagate_noalloc(c, M, &s, ldq, B, dt, steps, precision);
}

int lindblad_q_to_f32(lb_ctx* c, int64_t M, const double* Q, int64_t ldq, float* Q32) {
    CHECK_CTX(c);
    CHECK_PTR(Q);
    CHECK_PTR(Q32);
    if (M < 1 || ldq < M) return lb_fail(LB_ERR_INVALID_ARG, "bad sizes");
    return lb_impl_q_to_f32(c, M, Q, ldq, Q32);
}

int lindblad_propagate_csr(lb_ctx* c, int64_t M, const int64_t* rowptr, const int64_t* col, const double* val,
                           const double* K, double* V, int B, double dt, int64_t steps) {
    CHECK_CTX(c);
    CHECK_PTR(rowptr);
    CHECK_PTR(K);
    CHECK_PTR(V);
    if (M < 3) return lb_fail(LB_ERR_INVALID_ARG, "M too small");
    if (B < 1 || B > 64) return lb_fail(LB_ERR_INVALID_ARG, "B=%d out of range", B);
    if (!isfinite(dt) || steps < 0) return lb_fail(LB_ERR_INVALID_ARG, "bad dt/steps");
    return lb_impl_propagate_csr(c, M, rowptr, col, val, K, V, B, dt, steps);
}

int lindblad_propagate_csr_drive(lb_ctx* c, int64_t M, const int64_t* rowptr0, const int64_t* col0,
                                 const double* val0, const int64_t* rowptr1, const int64_t* col1, const double* val1,
                                 const double* K, double* V, int B, double dt, int64_t steps, double t0, int64_t k0,
                                 double E, double A, double T) {
    CHECK_CTX(c);
    CHECK_PTR(rowptr0);
    CHECK_PTR(rowptr1);
    CHECK_PTR(K);
    CHECK_PTR(V);
    if (M < 3) return lb_fail(LB_ERR_INVALID_ARG, "M too small");
    if (B < 1 || B > 64) return lb_fail(LB_ERR_INVALID_ARG, "B=%d out of range", B);
    if (!isfinite(dt) || steps < 0) return lb_fail(LB_ERR_INVALID_ARG, "bad dt/steps");
    if (!isfinite(t0) || !isfinite(E) || !isfinite(A) || !(T > 0) || !isfinite(T) || k0 < 0)
        return lb_fail(LB_ERR_INVALID_ARG, "drive needs finite t0, E, A, a period T > 0 and k0 >= 0");
    if (steps > 0) {
        // the drive switches at every multiple of T/2; each must fall on the step
        // grid t0 + k dt, so that every RK4 step integrates one constant system
        const double h = 0.5 * T / dt, ph = t0 / dt;
        const double rh = nearbyint(h), rph = nearbyint(ph);
        if (!(dt != 0) || !isfinite(h) || fabs(rh) < 1 || !(fabs(h - rh) <= 1e-9 * fabs(h)) ||
            !(fabs(ph - rph) <= 1e-9 * fmax(1.0, fabs(ph))))
            return lb_fail(LB_ERR_INVALID_ARG,
                           "the drive's switches (multiples of T/2) must fall on the step grid t0 + k dt: "
                           "T/(2 dt) = %.17g and t0/dt = %.17g must be integers (relative tolerance 1e-9)", h, ph);
    }
    return lb_impl_propagate_csr_drive(c, M, rowptr0, col0, val0, rowptr1, col1, val1, K, V, B, dt, steps, t0, k0, E,
                                       A, T);
}

int lb_read_bandwidth(lb_ctx* c, size_t bytes, double* gbs) {
    CHECK_CTX(c);
    CHECK_PTR(gbs);
    if (bytes < ((size_t)1 << 20)) return lb_fail(LB_ERR_INVALID_ARG, "probe needs at least 1 MiB");
    return lb_impl_read_bandwidth(c, bytes, gbs);
}

int lb_gemm_f64(lb_ctx* c, int trans_a, int trans_b, int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc) {
    CHECK_CTX(c);
    return lb_impl_gemm_f64(c->stream, trans_a != 0, trans_b != 0, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

int lb_gemm_c128(lb_ctx* c, int conj_a, int conj_b, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                 const double* B, int64_t ldb, double* C, int64_t ldc, double* work, int64_t work_elems) {
    CHECK_CTX(c);
    return lb_impl_gemm_c128(c->stream, conj_a != 0, conj_b != 0, m, n, k, A, lda, B, ldb, C, ldc, work, work_elems);
}

int lb_hessenberg(lb_ctx* c, int64_t M, double* A, int64_t lda) {
    CHECK_CTX(c);
    CHECK_PTR(A);
    if (M < 1 || M > LB_SPECTRUM_MAX_M) return lb_fail(LB_ERR_INVALID_ARG, "M out of range [1, %d]", LB_SPECTRUM_MAX_M);
    if (lda < M) return lb_fail(LB_ERR_INVALID_ARG, "lda < M");
    return lb_impl_hessenberg(c, (int)M, A, lda);
}

int lindblad_spectrum(lb_ctx* c, int64_t M, const double* Q, int64_t ldq, double* lam, lb_spectrum_info* info) {
    CHECK_CTX(c);
    CHECK_PTR(Q);
    CHECK_PTR(lam);
    if (M < 1 || M > LB_SPECTRUM_MAX_M) return lb_fail(LB_ERR_INVALID_ARG, "M out of range [1, %d]", LB_SPECTRUM_MAX_M);
    if (ldq < M) return lb_fail(LB_ERR_INVALID_ARG, "ldq < M");
    lb_spectrum_info counts = {};
    const int rc = lb_impl_spectrum(c, (int)M, Q, ldq, lam, &counts);
    if (info) *info = counts;
    return rc;
}

int lindblad_spectrum_histogram(lb_ctx* c, int64_t n, const double* lam, double re0, double re1, double im0,
                                double im1, int nx, int ny, int64_t* counts) {
    CHECK_CTX(c);
    CHECK_PTR(counts);
    if (n < 0 || (n > 0 && !lam)) return lb_fail(LB_ERR_INVALID_ARG, "bad n or null lam");
    if (nx < 1 || ny < 1 || (int64_t)nx * ny > ((int64_t)1 << 26))
        return lb_fail(LB_ERR_INVALID_ARG, "grid %d x %d out of range", nx, ny);
    if (!std::isfinite(re0) || !std::isfinite(re1) || !std::isfinite(im0) || !std::isfinite(im1) || !(re1 > re0) ||
        !(im1 > im0))
        return lb_fail(LB_ERR_INVALID_ARG, "grid bounds must be finite with re1 > re0 and im1 > im0");
    return lb_impl_spectrum_histogram(c, n, lam, re0, re1, im0, im1, nx, ny, counts);
}

static int system_args(const lb_system* sys) {
    if (!sys) return lb_fail(LB_ERR_INVALID_ARG, "null system");
    if (sys->N < 2 || sys->N > LB_MAX_N) return lb_fail(LB_ERR_INVALID_ARG, "N=%d out of range", sys->N);
    const int64_t M = (int64_t)sys->N * sys->N - 1;
    if (!sys->K) return lb_fail(LB_ERR_INVALID_ARG, "null K");
    if (sys->kind == LB_SYSTEM_DENSE) {
        if (!sys->Q) return lb_fail(LB_ERR_INVALID_ARG, "null Q");
        if (sys->ldq < M) return lb_fail(LB_ERR_INVALID_ARG, "ldq < M");
    } else if (sys->kind == LB_SYSTEM_CSR) {
        if (!sys->rowptr || sys->nnz < 0 || (sys->nnz > 0 && (!sys->col || !sys->val)))
            return lb_fail(LB_ERR_INVALID_ARG, "bad CSR");
    } else {
        return lb_fail(LB_ERR_INVALID_ARG, "unknown kind %d", sys->kind);
    }
    return LB_OK;
}

int lindblad_save_system(lb_ctx* c, const char* path, const lb_system* sys) {
    CHECK_CTX(c);
    CHECK_PTR(path);
    int rc = system_args(sys);
    if (rc) return rc;
    return lb_impl_save_system(c, path, sys);
}

int lindblad_load_system_info(const char* path, lb_system* sys) {
    CHECK_PTR(path);
    CHECK_PTR(sys);
    return lb_impl_load_system_info(path, sys);
}

int lindblad_load_system(lb_ctx* c, const char* path, lb_system* sys) {
    CHECK_CTX(c);
    CHECK_PTR(path);
    int rc = system_args(sys);
    if (rc) return rc;
    return lb_impl_load_system(c, path, sys);
}

int lb_eigh(lb_ctx* c, int N, double* A, int lda, double* w, double* Z, int ldz, int* sweeps) {
    CHECK_CTX(c);
    CHECK_PTR(A);
    CHECK_PTR(w);
    CHECK_PTR(Z);
    if (N < 1 || N > LB_MAX_N || lda < N || ldz < N) return lb_fail(LB_ERR_INVALID_ARG, "bad sizes");
    return lb_impl_eigh(c, N, A, lda, w, Z, ldz, sweeps);
}

static int steady_args(int64_t M, const double* K, const double* v, double tol, int64_t maxit, int64_t restart) {
    if (!K || !v) return lb_fail(LB_ERR_INVALID_ARG, "null pointer");
    if (M < 3) return lb_fail(LB_ERR_INVALID_ARG, "M too small");
    if (!(tol > 0 && tol < 1)) return lb_fail(LB_ERR_INVALID_ARG, "tol must lie in (0, 1)");
    if (maxit < 1 || restart < 1 || restart > 8192)
        return lb_fail(LB_ERR_INVALID_ARG, "maxit >= 1 and 1 <= restart <= 8192 required");
    return LB_OK;
}

int lindblad_steady_state(lb_ctx* c, int64_t M, const double* Q, int64_t ldq, const double* K, const lb_secular* pre,
                          double* v, double tol, int64_t maxit, int64_t restart, lb_solve_info* info) {
    CHECK_CTX(c);
    CHECK_PTR(Q);
    int rc = steady_args(M, K, v, tol, maxit, restart);
    if (rc) return rc;
    if (ldq < M) return lb_fail(LB_ERR_INVALID_ARG, "ldq < M");
    if (pre && lb_secular_size(pre) != M) return lb_fail(LB_ERR_INVALID_ARG, "preconditioner is for another M");
    lb_solve_info local;
    return lb_impl_steady_dense(c, M, Q, ldq, K, pre, v, tol, maxit, restart, info ? info : &local);
}

int lindblad_steady_state_csr(lb_ctx* c, int64_t M, const int64_t* rowptr, const int64_t* col, const double* val,
                              const double* K, const lb_secular* pre, double* v, double tol, int64_t maxit,
                              int64_t restart, lb_solve_info* info) {
    CHECK_CTX(c);
    CHECK_PTR(rowptr);
    int rc = steady_args(M, K, v, tol, maxit, restart);
    if (rc) return rc;
    if (pre && lb_secular_size(pre) != M) return lb_fail(LB_ERR_INVALID_ARG, "preconditioner is for another M");
    lb_solve_info local;
    return lb_impl_steady_csr(c, M, rowptr, col, val, K, pre, v, tol, maxit, restart, info ? info : &local);
}

int lindblad_secular_create(lb_ctx* c, int N, const lb_csr_c128* H, int P, const double* rates, const lb_csr_c128* L,
                            lb_secular** out) {
    CHECK_CTX(c);
    CHECK_PTR(H);
    CHECK_PTR(out);
    *out = nullptr;
    if (N < 2 || N > LB_MAX_N) return lb_fail(LB_ERR_INVALID_ARG, "N=%d out of range", N);
    if (P < 0 || (P > 0 && (!rates || !L))) return lb_fail(LB_ERR_INVALID_ARG, "bad jump operators");
    if (!H->rowptr || (H->nnz > 0 && (!H->col || !H->val))) return lb_fail(LB_ERR_INVALID_ARG, "bad H");
    for (int p = 0; p < P; ++p) {
        if (!(rates[p] >= 0) || !isfinite(rates[p])) return lb_fail(LB_ERR_INVALID_ARG, "rate %d not >= 0", p);
        if (!L[p].rowptr || (L[p].nnz > 0 && (!L[p].col || !L[p].val)))
            return lb_fail(LB_ERR_INVALID_ARG, "bad jump operator %d", p);
    }
    return lb_impl_secular_create(c, N, H, P, rates, L, out);
}

int lindblad_secular_destroy(lb_secular* pre) {
    lb_impl_secular_destroy(pre);
    return LB_OK;
}

int lindblad_propagate_batched(lb_ctx* c, int R, int64_t M, const double* const* Q, const float* const* Q32,
                               int64_t ldq, const double* const* K, double* const* V, int B, double dt,
                               int64_t steps, int precision) {
    CHECK_CTX(c);
    int rc = check_prop(M, ldq, B, dt, steps, precision);
    if (rc) return rc;
    if (R < 1 || R > 65535) return lb_fail(LB_ERR_INVALID_ARG, "R=%d out of range", R);
    CHECK_PTR(K);
    CHECK_PTR(V);
    std::vector<lb_prop_sys> sys(R);
    for (int r = 0; r < R; ++r) {
        sys[r].Q = Q ? Q[r] : nullptr;
        sys[r].Q32 = Q32 ? Q32[r] : nullptr;
        sys[r].K = K[r];
        sys[r].V = V[r];
        if (!sys[r].K || !sys[r].V || (precision == LB_FP64 && !sys[r].Q) || (precision == LB_FP32 && !sys[r].Q32))
            return lb_fail(LB_ERR_INVALID_ARG, "null pointer for system %d", r);
    }
    return lb_impl_propagate(c, R, M, sys.data(), ldq, B, dt, steps, precision, nullptr);
}

int lindblad_propagate_graph(lb_ctx* c, int64_t M, const double* Q, const float* Q32, int64_t ldq, const double* K,
                             double* V, int B, double dt, int64_t steps, int precision) {
    CHECK_CTX(c);
    int rc = check_prop(M, ldq, B, dt, steps, precision);
    if (rc) return rc;
    CHECK_PTR(K);
    CHECK_PTR(V);
    if (precision == LB_FP64) CHECK_PTR(Q);
    else CHECK_PTR(Q32);
    lb_prop_sys s{Q, Q32, K, V};
    return lb_impl_propagate_graph(c, M, &s, ldq, B, dt, steps, precision);
}

int lindblad_graph_clear(lb_ctx* c, int* freed) {
    CHECK_CTX(c);
    LB_HIP(hipSetDevice(c->device));
    LB_HIP(hipStreamSynchronize(c->stream));  // a cached graph's last launch may still run
    const int n = (int)c->graphs.size();
    for (auto& kv : c->graphs) lb_graph_free(kv.second);
    c->graphs.clear();
    if (freed) *freed = n;
    return LB_OK;
}

int lindblad_autotune(lb_ctx* c, int64_t M, const double* Q, const float* Q32, int64_t ldq, const double* K,
                      double* V, int B, int precision) {
    CHECK_CTX(c);
    int rc = check_prop(M, ldq, B, 0.0, 0, precision);
    if (rc) return rc;
    CHECK_PTR(K);
    CHECK_PTR(V);
    if (precision == LB_FP64) CHECK_PTR(Q);
    else CHECK_PTR(Q32);
    lb_prop_sys s{Q, Q32, K, V};
    return lb_impl_autotune(c, M, &s, ldq, B, precision);
}

int lindblad_time_stage(lb_ctx* c, int R, int64_t M, const double* const* Q, const float* const* Q32, int64_t ldq,
                        const double* const* K, double* const* V, int B, int precision, int iters, double* avg_ms) {
    CHECK_CTX(c);
    int rc = check_prop(M, ldq, B, 0.0, 0, precision);
    if (rc) return rc;
    if (R < 1 || R > 65535 || iters < 1) return lb_fail(LB_ERR_INVALID_ARG, "bad R or iters");
    CHECK_PTR(K);
    CHECK_PTR(V);
    CHECK_PTR(avg_ms);
    std::vector<lb_prop_sys> sys(R);
    for (int r = 0; r < R; ++r) {
        sys[r].Q = Q ? Q[r] : nullptr;
        sys[r].Q32 = Q32 ? Q32[r] : nullptr;
        sys[r].K = K[r];
        sys[r].V = V[r];
        if (!sys[r].K || !sys[r].V || (precision == LB_FP64 && !sys[r].Q) || (precision == LB_FP32 && !sys[r].Q32))
            return lb_fail(LB_ERR_INVALID_ARG, "null pointer for system %d", r);
    }
    return lb_impl_time_stage(c, R, M, sys.data(), ldq, B, precision, iters, avg_ms, nullptr);
}

int lindblad_set_tile(lb_ctx* c, int64_t M, int B, int precision, int rows, int kslab, int waves) {
    if (!c) return lb_fail(LB_ERR_INVALID_ARG, "null context");
    if (rows < 16 || rows % 16 || rows > 128 || kslab < 16 || kslab % 16 || waves < 1 || waves > 4)
        return lb_fail(LB_ERR_INVALID_ARG, "tile rows=%d kslab=%d waves=%d out of range", rows, kslab, waves);
    const int Bp = B <= 16 ? 16 : (B <= 32 ? 32 : 64);
    c->tuned[std::make_tuple(M, Bp, precision)] = lb_tile{rows, kslab, waves};
    return LB_OK;
}

int lindblad_tile_info(lb_ctx* c, int64_t M, int B, int precision, int* rows, int* kslab, int* waves, int* tuned) {
    if (!c) return lb_fail(LB_ERR_INVALID_ARG, "null context");
    const int Bp = B <= 16 ? 16 : (B <= 32 ? 32 : 64);
    auto it = c->tuned.find(std::make_tuple(M, Bp, precision));
    lb_tile t = it != c->tuned.end() ? it->second : lb_default_tile(M, Bp, precision, 1);
    if (rows) *rows = t.rows;
    if (kslab) *kslab = t.kslab;
    if (waves) *waves = t.waves;
    if (tuned) *tuned = it != c->tuned.end();
    return LB_OK;
}

}  // extern "C"
