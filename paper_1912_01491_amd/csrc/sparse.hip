// Sparse data preparation (placeholder until the CSR assembly lands).
#include "lb_internal.h"

int lb_impl_sparse(lb_ctx* c, int N, const lb_csr_c128* H, int P, const double* rates, const lb_csr_c128* L,
                   int64_t* nnz, int64_t* rowptr, int64_t* col, double* val, double* K) {
    (void)c; (void)N; (void)H; (void)P; (void)rates; (void)L; (void)nnz; (void)rowptr; (void)col; (void)val; (void)K;
    return lb_fail(LB_ERR_UNSUPPORTED, "sparse preparation not built");
}

