// Saving and loading a prepared system (Q, K): the paper prepares the ODE
// system once and runs the integration from stored data (Sec. 5), and a
// serving process can load systems another process prepared.
//
// File layout (little-endian, as the host writes it):
//   header (80 bytes): magic "LBSYSTEM", version 1, kind (0 dense, 1 CSR), N,
//   M, nnz (CSR; 0 for dense), payload hash, reserved;
//   dense payload: Q as M rows of M doubles (compact, whatever ldq the caller
//   used), then K (M doubles);
//   CSR payload: rowptr (M + 1 int64), col (nnz int64), val (nnz doubles), K.
// The hash is the wrap-around sum over the payload's 8-byte words w_i of
// mix(w_i xor i * 0x9E3779B97F4A7C15), mix being the SplitMix64 finaliser,
// computed on the device; it is order-independent, so any reduction order gives
// the same value, and position-sensitive through i. Loading recomputes it.
// Transfers go through two pinned 64 MB staging buffers so that the copy of
// one chunk overlaps the file I/O of the other.
#include "lb_internal.h"

#include <stdio.h>
#include <string.h>

namespace {

constexpr char kMagic[8] = {'L', 'B', 'S', 'Y', 'S', 'T', 'E', 'M'};
constexpr uint32_t kVersion = 1;
constexpr size_t kChunk = (size_t)64 << 20;

struct FileHeader {
    char magic[8];
    uint32_t version;
    uint32_t kind;
    int64_t N, M, nnz;
    uint64_t hash;
    uint64_t reserved[4];
};
static_assert(sizeof(FileHeader) == 80, "file header is 80 bytes");

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// out += sum over rows r < nrows of the row's first ncols words, word index
// base + r * ncols + c (rows ld words apart in memory).
__global__ __launch_bounds__(256) void k_hash(const uint64_t* a, int64_t nrows, int64_t ncols, int64_t ld,
                                              uint64_t base, unsigned long long* out) {
    __shared__ uint64_t red[4];
    const int64_t n = nrows * ncols;
    uint64_t s = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / ncols, c = i - r * ncols;
        s += mix64(a[r * ld + c] ^ ((base + (uint64_t)i) * 0x9E3779B97F4A7C15ull));
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, (unsigned long long)(red[0] + red[1] + red[2] + red[3]));
}

struct Part {  // one payload array as rows of words
    const void* dev;
    int64_t nrows, ncols, ld;  // in 8-byte words
};

static int parts_of(const lb_system* sys, int64_t M, Part* p, int* np) {
    if (sys->kind == LB_SYSTEM_DENSE) {
        p[0] = {sys->Q, M, M, sys->ldq};
        p[1] = {sys->K, 1, M, M};
        *np = 2;
    } else {
        p[0] = {sys->rowptr, 1, M + 1, M + 1};
        p[1] = {sys->col, 1, sys->nnz, sys->nnz};
        p[2] = {sys->val, 1, sys->nnz, sys->nnz};
        p[3] = {sys->K, 1, M, M};
        *np = 4;
    }
    return LB_OK;
}

static int device_hash(lb_ctx* c, const Part* p, int np, uint64_t* hash) {
    hipStream_t s = c->stream;
    int rc = lb_ws_reserve(c, 256);
    if (rc) return rc;
    unsigned long long* acc = (unsigned long long*)c->ws;
    LB_HIP(hipMemsetAsync(acc, 0, sizeof(unsigned long long), s));
    uint64_t base = 0;
    for (int k = 0; k < np; ++k) {
        const int64_t n = p[k].nrows * p[k].ncols;
        if (n > 0) {
            const unsigned grid = (unsigned)std::min<int64_t>(4096, lb_blocks(n, 256));
            hipLaunchKernelGGL(k_hash, dim3(grid), dim3(256), 0, s, (const uint64_t*)p[k].dev, p[k].nrows, p[k].ncols,
                               p[k].ld, base, acc);
            LB_CHECK_LAUNCH();
        }
        base += (uint64_t)n;
    }
    unsigned long long h = 0;
    LB_HIP(hipMemcpyAsync(&h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
    LB_HIP(hipStreamSynchronize(s));
    *hash = (uint64_t)h;
    return LB_OK;
}

// Two pinned staging buffers of kChunk bytes, freed on exit.
struct Staging {
    void* buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    ~Staging() {
        for (int i = 0; i < 2; ++i) {
            if (ev[i]) (void)hipEventDestroy(ev[i]);
            if (buf[i]) (void)hipHostFree(buf[i]);
        }
    }
    int init() {
        for (int i = 0; i < 2; ++i) {
            if (hipHostMalloc(&buf[i], kChunk, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                buf[i] = nullptr;
                return lb_fail(LB_ERR_OOM, "pinned staging buffer of %zu bytes", kChunk);
            }
            if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) {
                ev[i] = nullptr;
                return lb_fail(LB_ERR_DEVICE, "event creation failed");
            }
        }
        return LB_OK;
    }
};

struct FileCloser {
    FILE* f = nullptr;
    ~FileCloser() {
        if (f) fclose(f);
    }
};

// Streams one part (rows of ncols words, ld apart on the device) to the file:
// chunks of whole rows, or pieces of a row when one row exceeds a chunk.
static int write_part(lb_ctx* c, Staging& st, FILE* f, const Part& p) {
    hipStream_t s = c->stream;
    const size_t rowb = (size_t)p.ncols * 8;
    if (rowb == 0 || p.nrows == 0) return LB_OK;
    const int64_t rows_per = std::max<int64_t>(1, (int64_t)(kChunk / rowb));
    // enumerate pieces: (row0, rows, byte offset in row, bytes per row)
    struct Piece {
        int64_t r0, nr;
        size_t off, w;
    };
    std::vector<Piece> pieces;
    if (rowb <= kChunk) {
        for (int64_t r = 0; r < p.nrows; r += rows_per) pieces.push_back({r, std::min(rows_per, p.nrows - r), 0, rowb});
    } else {
        for (int64_t r = 0; r < p.nrows; ++r)
            for (size_t o = 0; o < rowb; o += kChunk) pieces.push_back({r, 1, o, std::min(kChunk, rowb - o)});
    }
    const char* base = (const char*)p.dev;
    auto issue = [&](size_t k) -> int {
        const Piece& q = pieces[k];
        const int b = (int)(k & 1);
        LB_HIP(hipMemcpy2DAsync(st.buf[b], q.w, base + (size_t)q.r0 * p.ld * 8 + q.off, (size_t)p.ld * 8, q.w,
                                (size_t)q.nr, hipMemcpyDeviceToHost, s));
        LB_HIP(hipEventRecord(st.ev[b], s));
        return LB_OK;
    };
    int rc = issue(0);
    if (rc) return rc;
    for (size_t k = 0; k < pieces.size(); ++k) {
        if (k + 1 < pieces.size() && (rc = issue(k + 1))) return rc;
        const int b = (int)(k & 1);
        LB_HIP(hipEventSynchronize(st.ev[b]));
        const size_t bytes = pieces[k].w * (size_t)pieces[k].nr;
        if (fwrite(st.buf[b], 1, bytes, f) != bytes) return lb_fail(LB_ERR_IO, "write failed");
        // the next issue reuses buffer b only after this write: issue(k + 2) happens in iteration k + 1
    }
    return LB_OK;
}

static int read_part(lb_ctx* c, Staging& st, FILE* f, const Part& p) {
    hipStream_t s = c->stream;
    const size_t rowb = (size_t)p.ncols * 8;
    if (rowb == 0 || p.nrows == 0) return LB_OK;
    const int64_t rows_per = std::max<int64_t>(1, (int64_t)(kChunk / rowb));
    char* base = (char*)p.dev;
    int b = 0;
    auto piece = [&](int64_t r0, int64_t nr, size_t off, size_t w) -> int {
        // the buffer's previous copy must have finished before it is refilled
        LB_HIP(hipEventSynchronize(st.ev[b]));
        const size_t bytes = w * (size_t)nr;
        if (fread(st.buf[b], 1, bytes, f) != bytes) return lb_fail(LB_ERR_IO, "file is shorter than its header says");
        LB_HIP(hipMemcpy2DAsync(base + (size_t)r0 * p.ld * 8 + off, (size_t)p.ld * 8, st.buf[b], w, w, (size_t)nr,
                                hipMemcpyHostToDevice, s));
        LB_HIP(hipEventRecord(st.ev[b], s));
        b ^= 1;
        return LB_OK;
    };
    int rc;
    if (rowb <= kChunk) {
        for (int64_t r = 0; r < p.nrows; r += rows_per)
            if ((rc = piece(r, std::min(rows_per, p.nrows - r), 0, rowb))) return rc;
    } else {
        for (int64_t r = 0; r < p.nrows; ++r)
            for (size_t o = 0; o < rowb; o += kChunk)
                if ((rc = piece(r, 1, o, std::min(kChunk, rowb - o)))) return rc;
    }
    return LB_OK;
}

static int read_header(FILE* f, FileHeader* h) {
    if (fread(h, 1, sizeof(*h), f) != sizeof(*h)) return lb_fail(LB_ERR_IO, "file too short for a header");
    if (memcmp(h->magic, kMagic, 8) != 0) return lb_fail(LB_ERR_IO, "not a saved system (bad magic)");
    if (h->version != kVersion) return lb_fail(LB_ERR_IO, "unsupported file version %u", h->version);
    if (h->kind > 1 || h->N < 2 || h->N > LB_MAX_N || h->M != h->N * h->N - 1 || h->nnz < 0 ||
        (h->kind == 0 && h->nnz != 0))
        return lb_fail(LB_ERR_IO, "inconsistent header");
    return LB_OK;
}

}  // namespace

int lb_impl_save_system(lb_ctx* c, const char* path, const lb_system* sys) {
    const int64_t M = (int64_t)sys->N * sys->N - 1;
    if (sys->kind == LB_SYSTEM_CSR) {  // the stored count must match the row pointers
        int64_t last = -1;
        LB_HIP(hipMemcpyAsync(&last, sys->rowptr + M, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
        LB_HIP(hipStreamSynchronize(c->stream));
        if (last != sys->nnz) return lb_fail(LB_ERR_INVALID_ARG, "rowptr[M] = %lld but nnz = %lld", (long long)last,
                                             (long long)sys->nnz);
    }
    Part p[4];
    int np = 0;
    parts_of(sys, M, p, &np);
    FileHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, kMagic, 8);
    h.version = kVersion;
    h.kind = sys->kind == LB_SYSTEM_DENSE ? 0 : 1;
    h.N = sys->N;
    h.M = M;
    h.nnz = sys->kind == LB_SYSTEM_DENSE ? 0 : sys->nnz;
    int rc = device_hash(c, p, np, &h.hash);
    if (rc) return rc;
    Staging st;
    if ((rc = st.init())) return rc;
    FileCloser fc;
    fc.f = fopen(path, "wb");
    if (!fc.f) return lb_fail(LB_ERR_IO, "cannot open %s for writing", path);
    if (fwrite(&h, 1, sizeof(h), fc.f) != sizeof(h)) return lb_fail(LB_ERR_IO, "write failed");
    for (int k = 0; k < np; ++k)
        if ((rc = write_part(c, st, fc.f, p[k]))) return rc;
    if (fflush(fc.f) != 0) return lb_fail(LB_ERR_IO, "write failed");
    return LB_OK;
}

int lb_impl_load_system_info(const char* path, lb_system* sys) {
    FileCloser fc;
    fc.f = fopen(path, "rb");
    if (!fc.f) return lb_fail(LB_ERR_IO, "cannot open %s", path);
    FileHeader h;
    int rc = read_header(fc.f, &h);
    if (rc) return rc;
    sys->kind = h.kind == 0 ? LB_SYSTEM_DENSE : LB_SYSTEM_CSR;
    sys->N = (int)h.N;
    sys->nnz = h.nnz;
    return LB_OK;
}

int lb_impl_load_system(lb_ctx* c, const char* path, lb_system* sys) {
    FileCloser fc;
    fc.f = fopen(path, "rb");
    if (!fc.f) return lb_fail(LB_ERR_IO, "cannot open %s", path);
    FileHeader h;
    int rc = read_header(fc.f, &h);
    if (rc) return rc;
    const int want = h.kind == 0 ? LB_SYSTEM_DENSE : LB_SYSTEM_CSR;
    if (sys->kind != want || sys->N != (int)h.N || (want == LB_SYSTEM_CSR && sys->nnz != h.nnz))
        return lb_fail(LB_ERR_INVALID_ARG, "buffers describe another system than the file (kind %d N %lld nnz %lld)",
                       want, (long long)h.N, (long long)h.nnz);
    if (want == LB_SYSTEM_DENSE && sys->ldq < h.M) return lb_fail(LB_ERR_INVALID_ARG, "ldq < M");
    Part p[4];
    int np = 0;
    parts_of(sys, h.M, p, &np);
    Staging st;
    if ((rc = st.init())) return rc;
    for (int k = 0; k < np; ++k)
        if ((rc = read_part(c, st, fc.f, p[k]))) return rc;
    if (want == LB_SYSTEM_DENSE && sys->ldq > h.M)  // padding columns zero, as lindblad_prepare leaves them
        LB_HIP(hipMemset2DAsync(sys->Q + h.M, (size_t)sys->ldq * 8, 0, (size_t)(sys->ldq - h.M) * 8, (size_t)h.M,
                                c->stream));
    uint64_t hash = 0;
    if ((rc = device_hash(c, p, np, &hash))) return rc;
    if (hash != h.hash) return lb_fail(LB_ERR_IO, "payload hash mismatch: the file is corrupt");
    return LB_OK;
}
