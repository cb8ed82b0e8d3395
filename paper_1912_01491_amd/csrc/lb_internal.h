// Internal declarations of the gfx950 library: context, workspace, error
// reporting, and device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lindblad.h"

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------

void lb_set_error(const char* fmt, ...);
int lb_fail(int code, const char* fmt, ...);

#define LB_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t _e = (call);                                                       \
        if (_e != hipSuccess)                                                         \
            return lb_fail(LB_ERR_DEVICE, "%s failed: %s (%s:%d)", #call,             \
                           hipGetErrorString(_e), __FILE__, __LINE__);                \
    } while (0)

#define LB_CHECK_LAUNCH()                                                             \
    do {                                                                              \
        hipError_t _e = hipGetLastError();                                            \
        if (_e != hipSuccess)                                                         \
            return lb_fail(LB_ERR_DEVICE, "kernel launch failed: %s (%s:%d)",         \
                           hipGetErrorString(_e), __FILE__, __LINE__);                \
    } while (0)

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------

struct lb_tile {
    int rows;   // rows per wave (multiple of 16)
    int kslab;  // columns per split-K slab (multiple of 16)
    int waves;  // waves per workgroup
};

struct lb_graph_key {
    int64_t M, ldq;
    int B, precision;
    const void *Q, *Q32, *K;
    double* V;
    double dt;
    int64_t steps;
    bool operator<(const lb_graph_key& o) const {
        return std::tie(M, ldq, B, precision, Q, Q32, K, V, dt, steps) <
               std::tie(o.M, o.ldq, o.B, o.precision, o.Q, o.Q32, o.K, o.V, o.dt, o.steps);
    }
};

struct lb_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    // growable workspace
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // pinned host scratch for small read-backs
    void* host = nullptr;
    size_t host_bytes = 0;
    // tuned tile shapes: key (M, Bp, precision)
    std::map<std::tuple<int64_t, int, int>, lb_tile> tuned;
    bool cache_loaded = false;
    // auxiliary stream for work that overlaps the context stream's (dense
    // preparation), joined back with events; created on first use
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // captured propagate graphs (at most 8, least recently used evicted)
    std::map<lb_graph_key, struct lb_graph_entry*> graphs;
    uint64_t graph_clock = 0;
    // progress of long calls (lb_set_progress)
    lb_progress_fn progress = nullptr;
    void* progress_user = nullptr;
};

// Calls the context's progress callback when one is set and about two seconds
// have passed since the last call (always for fraction 1 and for a new stage).
void lb_report(lb_ctx* c, const char* stage, double fraction);

struct lb_graph_entry;
void lb_graph_free(lb_graph_entry* g);

// Ensures the workspace holds at least `bytes`; returns LB_OK or LB_ERR_OOM.
int lb_ws_reserve(lb_ctx* c, size_t bytes);
int lb_host_reserve(lb_ctx* c, size_t bytes);

// Sets the current device to the context's device.
int lb_use_device(lb_ctx* c);

static inline size_t lb_align(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Basis helpers (host and device)
// ---------------------------------------------------------------------------

__host__ __device__ static inline int64_t lb_npairs(int N) { return (int64_t)N * (N - 1) / 2; }

// Position of the pair (j, k), j < k, in row-major pair order.
__host__ __device__ static inline int64_t lb_pair(int N, int j, int k) {
    return (int64_t)j * N - (int64_t)j * (j + 1) / 2 + (k - j - 1);
}

// Position of the unordered pair {a, b}, a != b.
__host__ __device__ static inline int64_t lb_upair(int N, int a, int b) {
    return a < b ? lb_pair(N, a, b) : lb_pair(N, b, a);
}

// Value of D^l at 0-based diagonal position x (l = 1..N-1).
__host__ __device__ static inline double lb_wdiag(int l, int x) {
    double nrm = 1.0 / sqrt((double)l * (double)(l + 1));
    return x < l ? nrm : (x == l ? -(double)l * nrm : 0.0);
}

// Basis position i -> (class 0 = S, 1 = J, 2 = D; j, k); for D, j = l, k = 0.
// Integer-exact: a floating estimate of the first pair vertex is corrected
// against the exact integer pair offsets.
__host__ __device__ static inline void lb_decode(int N, int64_t i, int& cls, int& j, int& k) {
    const int64_t P = lb_npairs(N);
    if (i >= 2 * P) {
        cls = 2;
        j = (int)(i - 2 * P) + 1;
        k = 0;
        return;
    }
    int64_t q = i;
    cls = 0;
    if (q >= P) {
        q -= P;
        cls = 1;
    }
    const double b = 2.0 * N - 1.0;
    int a = (int)floor((b - sqrt(b * b - 8.0 * (double)q)) * 0.5);
    a = a < 0 ? 0 : (a > N - 2 ? N - 2 : a);
    while (a > 0 && lb_pair(N, a, a + 1) > q) --a;
    while (a + 1 <= N - 2 && lb_pair(N, a + 1, a + 2) <= q) ++a;
    j = a;
    k = a + 1 + (int)(q - lb_pair(N, a, a + 1));
}

// ---------------------------------------------------------------------------
// Complex arithmetic on interleaved doubles
// ---------------------------------------------------------------------------

struct cd {
    double re, im;
};

__host__ __device__ static inline cd cmk(double r, double i) { return cd{r, i}; }
__host__ __device__ static inline cd cadd(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__host__ __device__ static inline cd csub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__host__ __device__ static inline cd cmul(cd a, cd b) {
    return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ static inline cd cconj(cd a) { return cd{a.re, -a.im}; }
__host__ __device__ static inline cd cscale(cd a, double s) { return cd{a.re * s, a.im * s}; }
// multiply by -i*s for s = +-1
__host__ __device__ static inline cd cmis(cd a, double s) { return cd{s * a.im, -s * a.re}; }

__device__ static inline cd cload(const double* p, int64_t idx) {
    const double2 v = *reinterpret_cast<const double2*>(p + 2 * idx);
    return cd{v.x, v.y};
}
__device__ static inline void cstore(double* p, int64_t idx, cd v) {
    *reinterpret_cast<double2*>(p + 2 * idx) = make_double2(v.re, v.im);
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------

static inline unsigned lb_blocks(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }
// Leading dimension of the library's own Q buffers: M rounded up to 32 elements
// (128-byte aligned rows in FP64 and FP32).
static inline int64_t lb_default_ldq(int64_t M) { return (M + 31) / 32 * 32; }

// ---------------------------------------------------------------------------
// Entry points implemented in the kernel translation units
// ---------------------------------------------------------------------------

int lb_impl_basis_table(lb_ctx* c, int N, int32_t* table);
int lb_impl_fd_count(lb_ctx* c, int N, int which, int64_t* count, int64_t* offsets_dev);
int lb_impl_fd_fill(lb_ctx* c, int N, int which, const int64_t* offsets_dev, int32_t* mns, double* val);

int lb_impl_expand(lb_ctx* c, int N, int B, const double* A, double* a, double scale);
int lb_impl_expand_pure(lb_ctx* c, int N, int B, const double* psi, double* V);
int lb_impl_reconstruct(lb_ctx* c, int N, int B, const double* V, double* rho);
int lb_impl_prepare_dense(lb_ctx* c, int N, const double* H, const double* gamma, double* Q,
                          int64_t ldq, double* K);
int lb_impl_hermitian_check(lb_ctx* c, int64_t n, const double* A, double* maxdev, double* maxabs);

int lb_impl_sparse(lb_ctx* c, int N, const lb_csr_c128* H, int P, const double* rates,
                   const lb_csr_c128* L, int64_t* nnz, int64_t* rowptr, int64_t* col, double* val,
                   double* K);

struct lb_prop_sys {
    const double* Q;
    const float* Q32;
    const double* K;
    double* V;
};

int lb_scratch_init(int device);
int lb_impl_propagate_noalloc(lb_ctx* c, int64_t M, const lb_prop_sys* sys, int64_t ldq, int B, double dt,
                              int64_t steps, int precision);
int lb_impl_propagate(lb_ctx* c, int R, int64_t M, const lb_prop_sys* sys, int64_t ldq, int B,
                      double dt, int64_t steps, int precision, const lb_tile* force_tile);
int lb_impl_time_stage(lb_ctx* c, int R, int64_t M, const lb_prop_sys* sys, int64_t ldq, int B, int precision,
                       int iters, double* ms, const lb_tile* force_tile);
int lb_impl_propagate_graph(lb_ctx* c, int64_t M, const lb_prop_sys* sys, int64_t ldq, int B, double dt,
                            int64_t steps, int precision);
int lb_impl_autotune(lb_ctx* c, int64_t M, const lb_prop_sys* sys, int64_t ldq, int B, int precision);
int lb_impl_propagate_csr(lb_ctx* c, int64_t M, const int64_t* rowptr, const int64_t* col,
                          const double* val, const double* K, double* V, int B, double dt,
                          int64_t steps);
int lb_impl_propagate_csr_drive(lb_ctx* c, int64_t M, const int64_t* rowptr0, const int64_t* col0,
                                const double* val0, const int64_t* rowptr1, const int64_t* col1, const double* val1,
                                const double* K, double* V, int B, double dt, int64_t steps, double t0, int64_t k0,
                                double E, double A, double T);
int lb_impl_q_to_f32(lb_ctx* c, int64_t M, const double* Q, int64_t ldq, float* Q32);
int lb_impl_save_system(lb_ctx* c, const char* path, const lb_system* sys);
int lb_impl_load_system_info(const char* path, lb_system* sys);
int lb_impl_load_system(lb_ctx* c, const char* path, lb_system* sys);
int lb_impl_read_bandwidth(lb_ctx* c, size_t bytes, double* gbs);
int lb_impl_eigh(lb_ctx* c, int N, double* A, int lda, double* w, double* Z, int ldz, int* sweeps);
int lb_impl_hessenberg(lb_ctx* c, int M, double* A, int64_t lda);
// FP64 matrix-core products (gemm.hip), column-major, asynchronous on s.
int lb_impl_gemm_f64(hipStream_t s, bool ta, bool tb, int64_t m, int64_t n, int64_t k, double alpha,
                     const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                     int64_t ldc);
// work: optional device scratch of work_elems complex values; when it holds S
// partial products (S = lb_gemm_c128_splits, fewer if it does not) k is split
// over S slices that are summed in order.
int lb_impl_gemm_c128(hipStream_t s, bool ca, bool cb, int64_t m, int64_t n, int64_t k, const double* A,
                      int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc, double* work,
                      int64_t work_elems);
int lb_gemm_c128_splits(int64_t m, int64_t n, int64_t k);
int lb_impl_spectrum(lb_ctx* c, int M, const double* Q, int64_t ldq, double* lam, lb_spectrum_info* info);
// Creates the context's auxiliary stream and its fork/join events on first use.
int lb_aux_stream(lb_ctx* c);
int lb_impl_spectrum_histogram(lb_ctx* c, int64_t n, const double* lam, double re0, double re1, double im0,
                               double im1, int nx, int ny, int64_t* counts);
int lb_impl_steady_dense(lb_ctx* c, int64_t M, const double* Q, int64_t ldq, const double* K, const lb_secular* pre,
                         double* v, double tol, int64_t maxit, int64_t restart, lb_solve_info* info);
int lb_impl_steady_csr(lb_ctx* c, int64_t M, const int64_t* rowptr, const int64_t* col, const double* val,
                       const double* K, const lb_secular* pre, double* v, double tol, int64_t maxit, int64_t restart,
                       lb_solve_info* info);
int lb_impl_secular_create(lb_ctx* c, int N, const lb_csr_c128* H, int P, const double* rates, const lb_csr_c128* L,
                           lb_secular** out);
int lb_impl_secular_apply(lb_ctx* c, const lb_secular* pre, const double* r, double* z);
void lb_impl_secular_destroy(lb_secular* pre);
int64_t lb_secular_size(const lb_secular* pre);  // M of the system it was built for
lb_tile lb_default_tile(int64_t M, int Bp, int precision, int R);
