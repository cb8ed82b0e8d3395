// Sparse matrices in the slice layout used by the sparse RK4 stage and the
// steady-state operator.
//
// The CSR rows a caller passes are regrouped once per call into slices of 64
// consecutive rows (one wavefront, one row per lane), each slice stored entry-
// major: entry k of the slice's rows sits at [k * 64 + lane], padded to the
// slice's longest row with zero values whose column is the lane's own row. A
// wavefront's column and value loads are then full contiguous lines, no
// cross-lane reduction is needed, and entry k of neighbouring rows, which in
// the pair ordering are neighbouring pairs, tends to gather neighbouring x.
// Rows with more than kLongRow entries (the diagonal-generator rows and the
// rows coupled to them, ~N entries) are left out of the slices and take one
// block of 256 threads each, with a fixed-order block reduction.
//
// A second matrix (the drive term Q1 of a time-dependent system) can be
// regrouped alongside; its long rows are those of the first matrix.
#pragma once

#include "lb_internal.h"

namespace {

constexpr int kLongRow = 32;
constexpr int kSlice = 64;
constexpr int kChunk = 4;  // slice entries per lane loaded before their products

// Slice widths (as 64 * entries, later scanned into offsets), the long-row
// mask of each slice and the list of long rows. One wavefront per slice.
__global__ __launch_bounds__(256) void k_sell_widths(int64_t M, int64_t S, const int64_t* rowptr,
                                                     const int64_t* rowptr1, int64_t* off0, int64_t* off1,
                                                     uint64_t* lmask, int* longrows, int* nlong) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t sl = r / kSlice;
    if (sl >= S) return;  // whole wavefronts
    int64_t len0 = 0, len1 = 0;
    if (r < M) {
        len0 = rowptr[r + 1] - rowptr[r];
        if (rowptr1) len1 = rowptr1[r + 1] - rowptr1[r];
    }
    const bool lng = len0 > kLongRow;
    if (lng) {
        len0 = 0;
        len1 = 0;
        longrows[atomicAdd(nlong, 1)] = (int)r;
    }
    for (int o = kSlice / 2; o > 0; o >>= 1) {
        len0 = max(len0, (int64_t)__shfl_xor(len0, o, kSlice));
        len1 = max(len1, (int64_t)__shfl_xor(len1, o, kSlice));
    }
    const uint64_t mask = __ballot(lng);
    if ((r & (kSlice - 1)) == 0) {
        off0[sl] = kSlice * len0;
        off1[sl] = kSlice * len1;
        lmask[sl] = mask;
    }
}

// Exclusive scan of n sizes in place, total in a[n]; one block of 1024 threads.
__device__ void block_scan_inplace(int64_t n, int64_t* a, int64_t* part) {
    const int t = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t b0 = min(n, t * per), b1 = min(n, b0 + per);
    int64_t sum = 0;
    for (int64_t i = b0; i < b1; ++i) sum += a[i];
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int i = 0; i < 1024; ++i) {
            const int64_t v = part[i];
            part[i] = run;
            run += v;
        }
        a[n] = run;
    }
    __syncthreads();
    int64_t run = part[t];
    for (int64_t i = b0; i < b1; ++i) {
        const int64_t v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_sell_scan(int64_t S, int64_t* off0, int64_t* off1) {
    __shared__ int64_t part[1024];
    block_scan_inplace(S, off0, part);
    if (off1) block_scan_inplace(S, off1, part);
}

// One matrix into the slice layout: thread per row (rows past M and long rows
// are all padding).
__device__ __forceinline__ void sell_put(int64_t r, int64_t M, int64_t sl, bool lng, const int64_t* rowptr,
                                         const int64_t* col, const double* val, const int64_t* off, int* scol,
                                         double* sval) {
    const int64_t o = off[sl], w = (off[sl + 1] - o) / kSlice;
    int64_t e0 = 0, len = 0;
    if (r < M && !lng) {
        e0 = rowptr[r];
        len = rowptr[r + 1] - e0;
    }
    const int pad = (int)(r < M ? r : M - 1);
    const int lane = (int)(r & (kSlice - 1));
    for (int64_t k = 0; k < w; ++k) {
        const int64_t d = o + k * kSlice + lane;
        scol[d] = k < len ? (int)col[e0 + k] : pad;
        sval[d] = k < len ? val[e0 + k] : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_sell_fill(int64_t M, int64_t S, const uint64_t* lmask, const int64_t* rowptr,
                                                   const int64_t* col, const double* val, const int64_t* off0,
                                                   int* scol0, double* sval0, const int64_t* rowptr1,
                                                   const int64_t* col1, const double* val1, const int64_t* off1,
                                                   int* scol1, double* sval1) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t sl = r / kSlice;
    if (sl >= S) return;
    const bool lng = (lmask[sl] >> (r & (kSlice - 1))) & 1;
    sell_put(r, M, sl, lng, rowptr, col, val, off0, scol0, sval0);
    if (rowptr1) sell_put(r, M, sl, lng, rowptr1, col1, val1, off1, scol1, sval1);
}

// A matrix (and optionally a second one) in the slice layout, with the CSR it
// came from (read by the long rows).
struct SellMat {
    int64_t M, S;
    const int64_t* rowptr;
    const int64_t* col;
    const double* val;
    const int64_t* rowptr1;
    const int64_t* col1;
    const double* val1;
    const int64_t* off0;  // slice offsets, S + 1 each
    const int* scol0;
    const double* sval0;
    const int64_t* off1;
    const int* scol1;
    const double* sval1;
    const uint64_t* lmask;  // per slice: lanes whose row is long
    const int* longrows;
    int nlong;
    int nlong8;   // long-row blocks padded to a multiple of 8
    int per_xcd;  // slice groups (of four slices) per XCD; launch nlong8 + 8 * per_xcd blocks
    int ngroups;  // slice groups
    int contig;   // slice groups in one contiguous range per XCD (sell_work)
};

// Work item of this block: a long row (w < nlong) or the slice group
// w - nlong; -1 for padding. Workgroups go to the 8 XCDs round robin by block
// id. The long rows keep that order (they are the heavy items, spread over
// all XCDs). With contig the slice groups are remapped so that each XCD
// walks one contiguous range of rows, whose gathers of x fall in three
// windows of about M/8 doubles (the rows' own pairs, the partner block, the
// diagonal part); that pays while those fit in the XCD's 4 MB L2 (M up to
// about 1.4 million) and costs beyond, where the natural order, with all
// XCDs on neighbouring rows at a time, shares one moving window instead.
__device__ __forceinline__ int sell_work(const SellMat& m) {
    const int b = blockIdx.x;
    if (b < m.nlong8) return b < m.nlong ? b : -1;
    const int sb = b - m.nlong8;
    const int g = m.contig ? (sb & 7) * m.per_xcd + (sb >> 3) : sb;
    return g < m.ngroups ? m.nlong + g : -1;
}

// acc[j] += sum over slice entries [k, k + n) of value * x_j[column], in entry
// order, for the first nb of SB states; FULL: n == kChunk.
template <int SB, bool FULL>
__device__ __forceinline__ void sell_chunk(const int* c0, const double* v0, int k, int n, const double* Xin,
                                           int64_t M, int nb, double* acc) {
    int cc[kChunk];
    double vv[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u)
        if (FULL || u < n) {
            cc[u] = c0[(int64_t)(k + u) * kSlice];
            vv[u] = v0[(int64_t)(k + u) * kSlice];
        }
#pragma unroll
    for (int j = 0; j < SB; ++j)
        if (j < nb) {
            const double* x = Xin + (int64_t)j * M;
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
                if (FULL || u < n) acc[j] = fma(vv[u], x[cc[u]], acc[j]);
        }
}

template <int SB>
__device__ __forceinline__ void sell_row(const int* c0, const double* v0, int w, const double* Xin, int64_t M,
                                         int nb, double* acc) {
    int k = 0;
    for (; k + kChunk <= w; k += kChunk) sell_chunk<SB, true>(c0, v0, k, kChunk, Xin, M, nb, acc);
    if (k < w) sell_chunk<SB, false>(c0, v0, k, w - k, Xin, M, nb, acc);
}


// Sums of one long row of the matrix (s0) and of the second matrix (s1, when
// TWO) against x, by a block of 256 threads in a fixed order; every thread
// receives both.
template <bool TWO>
__device__ __forceinline__ void block_row_dots(const SellMat& m, int64_t row, const double* x, double& s0out,
                                               double& s1out) {
    __shared__ double red[4], red1[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t e0 = m.rowptr[row], e1 = m.rowptr[row + 1];
    double s0 = 0.0, s1 = 0.0;
    int64_t e = e0 + threadIdx.x;
    for (; e + 256 < e1; e += 512) {
        s0 = fma(m.val[e], x[m.col[e]], s0);
        s1 = fma(m.val[e + 256], x[m.col[e + 256]], s1);
    }
    if (e < e1) s0 = fma(m.val[e], x[m.col[e]], s0);
    double sum = s0 + s1;
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    double sd = 0.0;
    if (TWO) {
        for (int64_t f = m.rowptr1[row] + threadIdx.x; f < m.rowptr1[row + 1]; f += 256)
            sd = fma(m.val1[f], x[m.col1[f]], sd);
        for (int o = 32; o > 0; o >>= 1) sd += __shfl_xor(sd, o, 64);
    }
    if (lane == 0) {
        red[wave] = sum;
        red1[wave] = sd;
    }
    __syncthreads();
    s0out = (red[0] + red[1]) + (red[2] + red[3]);
    s1out = (red1[0] + red1[1]) + (red1[2] + red1[3]);
    __syncthreads();
}

// Regroups the CSR matrix (and the second one, if rowptr1 is not null) into
// the slice layout inside the context workspace, which is laid out as
// [slice offsets, masks, long rows | caller's region of extra_bytes | slices].
// On return c->ws + *extra_off is the caller's region (the workspace may have
// been reallocated, so pointers into it must be taken afterwards). Enqueued on
// the context stream; synchronises twice to learn the sizes.
static int sell_build(lb_ctx* c, int64_t M, const int64_t* rowptr, const int64_t* col, const double* val,
                      const int64_t* rowptr1, const int64_t* col1, const double* val1, size_t extra_bytes,
                      SellMat* out, size_t* extra_off) {
    hipStream_t s = c->stream;
    const bool two = rowptr1 != nullptr;
    // numbers of stored entries: 32-bit slice columns
    int64_t nnz = 0, nnz1 = 0;
    LB_HIP(hipMemcpyAsync(&nnz, rowptr + M, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (two) LB_HIP(hipMemcpyAsync(&nnz1, rowptr1 + M, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LB_HIP(hipStreamSynchronize(s));
    if (nnz < 0 || nnz >= ((int64_t)1 << 31) || nnz1 < 0 || nnz1 >= ((int64_t)1 << 31))
        return lb_fail(LB_ERR_UNSUPPORTED, "nnz=%lld / %lld out of range", (long long)nnz, (long long)nnz1);
    const int64_t S = (M + kSlice - 1) / kSlice;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = lb_align(off + (bytes > 0 ? bytes : 1), 256);
        return o;
    };
    // phase 1 (sizes known from M): slice offsets, long-row masks and list
    const size_t o_off0 = take(sizeof(int64_t) * (size_t)(S + 1));
    const size_t o_off1 = take(sizeof(int64_t) * (size_t)(S + 1));
    const size_t o_mask = take(sizeof(uint64_t) * (size_t)S);
    const size_t o_long = take(sizeof(int) * (size_t)M);
    const size_t o_nl = take(sizeof(int));
    const size_t o_extra = take(extra_bytes);
    const size_t fixed = off;
    int rc = lb_ws_reserve(c, fixed);
    if (rc) return rc;
    int hl = 0;
    int64_t tot0 = 0, tot1 = 0;
    const unsigned rgrid = (unsigned)lb_blocks(S * kSlice, 256);
    for (int pass = 0; pass < 2; ++pass) {
        char* ws = (char*)c->ws;
        int64_t* off0 = (int64_t*)(ws + o_off0);
        int64_t* off1 = (int64_t*)(ws + o_off1);
        int* nlong = (int*)(ws + o_nl);
        LB_HIP(hipMemsetAsync(nlong, 0, sizeof(int), s));
        hipLaunchKernelGGL(k_sell_widths, dim3(rgrid), dim3(256), 0, s, M, S, rowptr, two ? rowptr1 : nullptr, off0,
                           off1, (uint64_t*)(ws + o_mask), (int*)(ws + o_long), nlong);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_sell_scan, dim3(1), dim3(1024), 0, s, S, off0, two ? off1 : nullptr);
        LB_CHECK_LAUNCH();
        LB_HIP(hipMemcpyAsync(&hl, nlong, sizeof(int), hipMemcpyDeviceToHost, s));
        LB_HIP(hipMemcpyAsync(&tot0, off0 + S, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        if (two) LB_HIP(hipMemcpyAsync(&tot1, off1 + S, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        LB_HIP(hipStreamSynchronize(s));
        off = fixed;
        take(sizeof(int) * (size_t)tot0);
        take(sizeof(double) * (size_t)tot0);
        take(sizeof(int) * (size_t)tot1);
        take(sizeof(double) * (size_t)tot1);
        if (off <= c->ws_bytes) break;
        // the workspace grows: its contents go, so the offsets are formed again
        rc = lb_ws_reserve(c, off);
        if (rc) return rc;
    }
    off = fixed;
    const size_t o_sc0 = take(sizeof(int) * (size_t)tot0);
    const size_t o_sv0 = take(sizeof(double) * (size_t)tot0);
    const size_t o_sc1 = take(sizeof(int) * (size_t)tot1);
    const size_t o_sv1 = take(sizeof(double) * (size_t)tot1);
    if (off > c->ws_bytes) return lb_fail(LB_ERR_DEVICE, "slice layout exceeds the workspace");
    char* ws = (char*)c->ws;
    SellMat m;
    m.M = M;
    m.S = S;
    m.rowptr = rowptr;
    m.col = col;
    m.val = val;
    m.rowptr1 = two ? rowptr1 : nullptr;
    m.col1 = col1;
    m.val1 = val1;
    m.off0 = (const int64_t*)(ws + o_off0);
    m.scol0 = (const int*)(ws + o_sc0);
    m.sval0 = (const double*)(ws + o_sv0);
    m.off1 = (const int64_t*)(ws + o_off1);
    m.scol1 = (const int*)(ws + o_sc1);
    m.sval1 = (const double*)(ws + o_sv1);
    m.lmask = (const uint64_t*)(ws + o_mask);
    m.longrows = (const int*)(ws + o_long);
    m.nlong = hl;
    m.nlong8 = (hl + 7) / 8 * 8;
    m.ngroups = (int)((S + 3) / 4);
    m.per_xcd = (m.ngroups + 7) / 8;
    m.contig = 3 * 8 * (M / 8) <= ((int64_t)4 << 20);  // three windows of M/8 doubles within 4 MB
    hipLaunchKernelGGL(k_sell_fill, dim3(rgrid), dim3(256), 0, s, M, S, m.lmask, rowptr, col, val, m.off0,
                       (int*)(ws + o_sc0), (double*)(ws + o_sv0), two ? rowptr1 : nullptr, col1, val1, m.off1,
                       (int*)(ws + o_sc1), (double*)(ws + o_sv1));
    LB_CHECK_LAUNCH();
    *out = m;
    *extra_off = o_extra;
    return LB_OK;
}

}  // namespace
