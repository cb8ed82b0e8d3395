// Row dot products of a wavefront over a dense FP64 matrix: the inner loop of
// the one-state RK4 stage GEMV and of the dense steady-state operator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double lb_double2v __attribute__((ext_vector_type(2)));

namespace {

// acc[t] = sum_c qrow[t][c] x[c] for R rows, lanes along the row reading 16
// bytes each (one load instruction covers 1 KB of a row; with ALIGNED the rows
// are 16-byte aligned and x is read as pairs; with NT, Q is read with the
// nontemporal hint as it is streamed once), reduced across the wavefront so
// every lane holds all R sums. A row's sum does not depend on R.
template <int R, bool ALIGNED, bool NT>
__device__ __forceinline__ void wave_rowdots(const double* const* qrow, const double* x, int64_t M, int lane,
                                             double* acc) {
#pragma unroll
    for (int t = 0; t < R; ++t) acc[t] = 0.0;
    int64_t c = 2 * lane;
    if (ALIGNED) {
        // four column steps per round: their 4 (R + 1) loads issued before the products, which
        // then run in the same order as one step at a time
        for (; c + 3 * 128 + 1 < M; c += 4 * 128) {
            double2 xv[4];
            lb_double2v q[4][R];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xv[u] = *reinterpret_cast<const double2*>(x + c + u * 128);
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    const double* a = qrow[t] + c + u * 128;
                    if (NT) q[u][t] = __builtin_nontemporal_load((const lb_double2v __attribute__((address_space(1)))*)a);
                    else q[u][t] = *reinterpret_cast<const lb_double2v*>(a);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    acc[t] = fma(q[u][t].x, xv[u].x, acc[t]);
                    acc[t] = fma(q[u][t].y, xv[u].y, acc[t]);
                }
        }
        for (; c + 1 < M; c += 128) {
            const double2 xv = *reinterpret_cast<const double2*>(x + c);
#pragma unroll
            for (int t = 0; t < R; ++t) {
                lb_double2v q;
                if (NT) q = __builtin_nontemporal_load((const lb_double2v __attribute__((address_space(1)))*)(qrow[t] + c));
                else q = *reinterpret_cast<const lb_double2v*>(qrow[t] + c);
                acc[t] = fma(q.x, xv.x, acc[t]);
                acc[t] = fma(q.y, xv.y, acc[t]);
            }
        }
    } else {
        // the same rounds with 8-byte loads
        for (; c + 3 * 128 + 1 < M; c += 4 * 128) {
            double xv[4][2], q[4][R][2];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xv[u][0] = x[c + u * 128];
                xv[u][1] = x[c + u * 128 + 1];
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    q[u][t][0] = qrow[t][c + u * 128];
                    q[u][t][1] = qrow[t][c + u * 128 + 1];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    acc[t] = fma(q[u][t][0], xv[u][0], acc[t]);
                    acc[t] = fma(q[u][t][1], xv[u][1], acc[t]);
                }
        }
        for (; c + 1 < M; c += 128) {
            const double x0 = x[c], x1 = x[c + 1];
#pragma unroll
            for (int t = 0; t < R; ++t) {
                acc[t] = fma(qrow[t][c], x0, acc[t]);
                acc[t] = fma(qrow[t][c + 1], x1, acc[t]);
            }
        }
    }
    if (c < M) {
        const double x0 = x[c];
#pragma unroll
        for (int t = 0; t < R; ++t) acc[t] = fma(qrow[t][c], x0, acc[t]);
    }
#pragma unroll
    for (int t = 0; t < R; ++t) {
        double v = acc[t];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        acc[t] = v;
    }
}

}  // namespace
