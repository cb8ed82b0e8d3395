// Sparse data preparation (placeholder until the CSR assembly lands).
#include "lb_internal.h"

int lb_impl_sparse(lb_ctx* c, int N, const lb_csr_c128* H, int P, const double* rates, const lb_csr_c128* L,
                   int64_t* nnz, int64_t* rowptr, int64_t* col, double* val, double* K) {
    (void)c; (void)N; (void)H; (void)P; (void)rates; (void)L; (void)nnz; (void)rowptr; (void)col; (void)val; (void)K;
    return lb_fail(LB_ERR_UNSUPPORTED, "sparse preparation not built");
}

extern "C" int lindblad_autotune(lb_ctx* c, int64_t M, const double* Q, const float* Q32, int64_t ldq,
                                 const double* K, double* V, int B, int precision) {
    (void)c; (void)M; (void)Q; (void)Q32; (void)ldq; (void)K; (void)V; (void)B; (void)precision;
    return lb_fail(LB_ERR_UNSUPPORTED, "autotune not built");
}

extern "C" int lindblad_propagate_graph(lb_ctx* c, int64_t M, const double* Q, const float* Q32, int64_t ldq,
                                        const double* K, double* V, int B, double dt, int64_t steps, int precision) {
    return lindblad_propagate(c, M, Q, Q32, ldq, K, V, B, dt, steps, precision);
}
