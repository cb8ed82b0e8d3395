/*
 * lindblad_oracle.c -- plain, slow, FP64 CPU oracle for the GKSL -> real ODE
 * transformation and its RK4 integration.
 *
 * TEST INFRASTRUCTURE. This file is the reference the GPU library is checked
 * against. Only the test suite, the smoke check and the benchmark's CPU
 * baseline leg may load it; the GPU library never links, includes or calls it,
 * and the two share no code.
 *
 * Source: Meyerov, Kozinov, Liniov, Volokitin, Yusipov, Ivanchenko, Denisov,
 * "Transforming Lindblad Equations into Systems of Real-Valued Linear
 * Equations: Performance Optimization and Parallelization of an Algorithm"
 * (arXiv:1912.01491). Equation numbers count the displayed equations of
 * Sections 2-3 in order of appearance: (1) the Lindbladian, (2) its
 * dissipator, (3)-(5) the S, J, D generators, (6) the expansion of a
 * Hermitian matrix, (7) the coherence vector, (8) the rewritten dissipator,
 * (9) the expanded equation, (10) the real ODE, (11) f and d, (12) z,
 * (13) q, (14) k, (15) r, (16)-(17) the dimer model.
 *
 * Readings taken where the text is garbled or ambiguous (each one is pinned
 * by a brute-force or closed-form test):
 *  - D^l of Eq. (5) is read as (sum_{x<=l} e_x e_x^T - l e_{l+1} e_{l+1}^T)
 *    / sqrt(l(l+1)): Hermitian and orthonormal as Sec. 2 requires.
 *  - Basis order: the S block (pairs j<k, row-major), then the J block in the
 *    same pair order, then D^1..D^{N-1}; all indices 0-based.
 *  - The dissipator is sum_jk gamma_jk (F_j rho F_k - 1/2 {F_k F_j, rho}) with
 *    gamma = sum_p gamma_p l_p l_p^dagger, the form Eqs. (8), (14), (15) use.
 *  - Eq. (14) carries the sum over p (gamma_jk in place of l_j conj(l_k)).
 *  - Eq. (15) takes the prefactor -1/4 with f and d as defined in Eq. (11).
 *  - The identity part of a jump operator L = L0 + c 1 is moved into the
 *    Hamiltonian: H += (i g / 2)(conj(c) L0 - c L0^dagger).
 *
 * Structure constants are never tabulated from closed forms here: every
 * f_abc and d_abc is the expansion coefficient of the commutator /
 * anticommutator of two basis matrices (Eq. (11)), evaluated from sparse
 * matrix products. A coefficient whose magnitude is below ZERO_TOL is taken
 * as an exact zero (true nonzeros are at least ~1/N in magnitude).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ZERO_TOL 1e-9

/* ------------------------------------------------------------------------ */
/* Basis (Sec. 2, Eqs. (3)-(5))                                              */
/* ------------------------------------------------------------------------ */

static long n_pairs(int N) { return (long)N * (N - 1) / 2; }

/* pair (j,k), j<k, row-major position */
static long pair_pos(int N, int j, int k) {
    return (long)j * N - (long)j * (j + 1) / 2 + (k - j - 1);
}

long or_index_of(int N, int cls, int j, int k) {
    long P = n_pairs(N);
    if (cls == 0) return pair_pos(N, j, k);
    if (cls == 1) return P + pair_pos(N, j, k);
    return 2 * P + (j - 1); /* D^l with l = j */
}

/* i -> (cls, j, k); for D, j = l (1..N-1) and k = 0 */
static long pair_start(int N, int j) { return (long)j * N - (long)j * (j + 1) / 2; }

void or_class_of(int N, long i, int* cls, int* j, int* k) {
    long P = n_pairs(N);
    if (i >= 2 * P) { *cls = 2; *j = (int)(i - 2 * P) + 1; *k = 0; return; }
    long q = i;
    *cls = 0;
    if (q >= P) { q -= P; *cls = 1; }
    /* first vertex a: largest a with pair_start(a) <= q (estimate, then exact integer correction) */
    double b = 2.0 * N - 1.0;
    long a = (long)floor((b - sqrt(b * b - 8.0 * (double)q)) / 2.0);
    if (a < 0) a = 0;
    if (a > N - 2) a = N - 2;
    while (a > 0 && pair_start(N, (int)a) > q) a--;
    while (a + 1 <= N - 2 && pair_start(N, (int)a + 1) <= q) a++;
    *j = (int)a;
    *k = (int)a + 1 + (int)(q - pair_start(N, (int)a));
}

/* value of D^l at diagonal position r (0-based row), Eq. (5) as read above */
static double dval(int l, int r) {
    double nrm = 1.0 / sqrt((double)l * (double)(l + 1));
    if (r < l) return nrm;
    if (r == l) return -(double)l * nrm;
    return 0.0;
}

/* nonzero entries of F_i; returns count (<= N) */
static int basis_entries(int N, long i, int* r, int* c, cplx* v) {
    int cls, j, k;
    or_class_of(N, i, &cls, &j, &k);
    const double s = 1.0 / sqrt(2.0);
    if (cls == 0) {
        r[0] = j; c[0] = k; v[0] = s;
        r[1] = k; c[1] = j; v[1] = s;
        return 2;
    }
    if (cls == 1) { /* J^(j,k) = -i/sqrt2 (e_j e_k^T - e_k e_j^T) */
        r[0] = j; c[0] = k; v[0] = -I * s;
        r[1] = k; c[1] = j; v[1] = I * s;
        return 2;
    }
    int n = 0;
    for (int x = 0; x <= j; x++) { r[n] = x; c[n] = x; v[n] = dval(j, x); n++; }
    return n;
}

void or_basis_dense(int N, long i, double* F /* N*N complex interleaved */) {
    memset(F, 0, sizeof(double) * 2 * (size_t)N * N);
    int* r = malloc(sizeof(int) * N);
    int* c = malloc(sizeof(int) * N);
    cplx* v = malloc(sizeof(cplx) * N);
    int n = basis_entries(N, i, r, c, v);
    for (int t = 0; t < n; t++) {
        F[2 * ((size_t)r[t] * N + c[t])] = creal(v[t]);
        F[2 * ((size_t)r[t] * N + c[t]) + 1] = cimag(v[t]);
    }
    free(r); free(c); free(v);
}

/* ------------------------------------------------------------------------ */
/* Per-thread workspace for sparse products and expansions                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    int N;
    long M;
    cplx* C;              /* N*N: commutator accumulator     */
    cplx* A;              /* N*N: anticommutator accumulator */
    unsigned char* mark;  /* N*N: touched flags              */
    int* touched;         /* touched flat indices            */
    int nt;
    unsigned char* cmark; /* M: candidate flags              */
    long* cand;
    long ncand;
    int* er; int* ec; cplx* ev;     /* entries of F_a */
    int* fr; int* fc; cplx* fv;     /* entries of F_b */
    int* browcol; cplx* browval; unsigned char* brow; /* row map of F_b */
    int* arowcol; cplx* arowval; unsigned char* arow; /* row map of F_a */
    int* diag; int ndiag;
} ws_t;

static ws_t* ws_new(int N) {
    ws_t* w = calloc(1, sizeof(ws_t));
    w->N = N;
    w->M = (long)N * N - 1;
    size_t NN = (size_t)N * N;
    w->C = malloc(sizeof(cplx) * NN);
    w->A = malloc(sizeof(cplx) * NN);
    w->mark = calloc(NN, 1);
    w->touched = malloc(sizeof(int) * NN);
    w->cmark = calloc((size_t)w->M, 1);
    w->cand = malloc(sizeof(long) * (size_t)w->M);
    w->er = malloc(sizeof(int) * N); w->ec = malloc(sizeof(int) * N); w->ev = malloc(sizeof(cplx) * N);
    w->fr = malloc(sizeof(int) * N); w->fc = malloc(sizeof(int) * N); w->fv = malloc(sizeof(cplx) * N);
    w->browcol = malloc(sizeof(int) * N); w->browval = malloc(sizeof(cplx) * N); w->brow = calloc(N, 1);
    w->arowcol = malloc(sizeof(int) * N); w->arowval = malloc(sizeof(cplx) * N); w->arow = calloc(N, 1);
    w->diag = malloc(sizeof(int) * N);
    return w;
}

static void ws_free(ws_t* w) {
    free(w->C); free(w->A); free(w->mark); free(w->touched); free(w->cmark); free(w->cand);
    free(w->er); free(w->ec); free(w->ev); free(w->fr); free(w->fc); free(w->fv);
    free(w->browcol); free(w->browval); free(w->brow);
    free(w->arowcol); free(w->arowval); free(w->arow);
    free(w->diag);
    free(w);
}

static void touch(ws_t* w, int idx) {
    if (!w->mark[idx]) { w->mark[idx] = 1; w->touched[w->nt++] = idx; w->C[idx] = 0; w->A[idx] = 0; }
}

static void ws_clear(ws_t* w) {
    for (int t = 0; t < w->nt; t++) w->mark[w->touched[t]] = 0;
    w->nt = 0;
}

/* Does F_a share a row/column index with F_b (so that a product can be nonzero)? */
static void support(int N, long i, int* lo, int* hi, int* isdiag, int* p, int* q) {
    int cls, j, k;
    or_class_of(N, i, &cls, &j, &k);
    if (cls == 2) { *isdiag = 1; *lo = 0; *hi = j; *p = -1; *q = -1; }
    else { *isdiag = 0; *lo = j; *hi = k; *p = j; *q = k; }
}

static int overlap(int N, long a, long b) {
    int lo1, hi1, d1, p1, q1, lo2, hi2, d2, p2, q2;
    support(N, a, &lo1, &hi1, &d1, &p1, &q1);
    support(N, b, &lo2, &hi2, &d2, &p2, &q2);
    if (d1 && d2) return 1;
    if (d1) return (p2 <= hi1) || (q2 <= hi1);
    if (d2) return (p1 <= hi2) || (q1 <= hi2);
    return p1 == p2 || p1 == q2 || q1 == p2 || q1 == q2;
}

/* list of basis elements whose support meets that of F_a (candidates b with F_a F_b or F_b F_a != 0) */
static long overlap_list(int N, long a, long* out) {
    long n = 0;
    long P = n_pairs(N);
    int lo, hi, isd, p, q;
    support(N, a, &lo, &hi, &isd, &p, &q);
    if (isd) {
        /* D^l (support rows 0..l) meets every pair (u,v) with u <= l and every D */
        for (int u = 0; u <= hi && u < N - 1; u++)
            for (int v = u + 1; v < N; v++) { long pp = pair_pos(N, u, v); out[n++] = pp; out[n++] = P + pp; }
        for (int l = 1; l < N; l++) out[n++] = 2 * P + (l - 1);
        return n;
    }
    /* pairs touching p or q */
    int vs[2] = {p, q};
    for (int t = 0; t < 2; t++) {
        int x = vs[t];
        for (int y = 0; y < N; y++) {
            if (y == x) continue;
            int u = x < y ? x : y, v = x < y ? y : x;
            if (t == 1 && (u == p && v == q)) continue; /* pair (p,q) already listed */
            long pp = pair_pos(N, u, v);
            out[n++] = pp;
            out[n++] = P + pp;
        }
    }
    /* diagonal generators D^l (support 0..l) meeting p or q: l >= p */
    for (int l = (p > 1 ? p : 1); l < N; l++) out[n++] = 2 * P + (l - 1);
    return n;
}

/*
 * fiber(a, b): all c with f_abc != 0 or d_abc != 0 (Eq. (11)):
 *   f_abc = -i Tr(F_c [F_a, F_b]),   d_abc = Tr(F_c {F_a, F_b}).
 * Computed by forming the sparse products F_a F_b and F_b F_a and reading
 * off the expansion coefficients Tr(F_c X) from the entries of F_c.
 * need_d = 0 skips the anticommutator (d returned as 0).
 * Returns the number of entries written to (c_out, f_out, d_out).
 */
static long fiber(ws_t* w, long a, long b, int need_d, long* c_out, double* f_out, double* d_out) {
    int N = w->N;
    long P = n_pairs(N);
    int na = basis_entries(N, a, w->er, w->ec, w->ev);
    int nb = basis_entries(N, b, w->fr, w->fc, w->fv);
    /* row maps: each basis matrix has at most one entry per row */
    for (int t = 0; t < nb; t++) { w->brow[w->fr[t]] = 1; w->browcol[w->fr[t]] = w->fc[t]; w->browval[w->fr[t]] = w->fv[t]; }
    for (int t = 0; t < na; t++) { w->arow[w->er[t]] = 1; w->arowcol[w->er[t]] = w->ec[t]; w->arowval[w->er[t]] = w->ev[t]; }
    /* F_a F_b */
    for (int t = 0; t < na; t++) {
        int r1 = w->er[t], c1 = w->ec[t];
        if (!w->brow[c1]) continue;
        int idx = r1 * N + w->browcol[c1];
        cplx pv = w->ev[t] * w->browval[c1];
        touch(w, idx);
        w->C[idx] += pv;
        w->A[idx] += pv;
    }
    /* F_b F_a */
    for (int t = 0; t < nb; t++) {
        int r1 = w->fr[t], c1 = w->fc[t];
        if (!w->arow[c1]) continue;
        int idx = r1 * N + w->arowcol[c1];
        cplx pv = w->fv[t] * w->arowval[c1];
        touch(w, idx);
        w->C[idx] -= pv;
        w->A[idx] += pv;
    }
    for (int t = 0; t < nb; t++) w->brow[w->fr[t]] = 0;
    for (int t = 0; t < na; t++) w->arow[w->er[t]] = 0;

    /* candidates c: pairs at touched off-diagonal positions, D^l at touched diagonal ones */
    w->ncand = 0;
    w->ndiag = 0;
    int mindiag = N;
    for (int t = 0; t < w->nt; t++) {
        int idx = w->touched[t];
        cplx cv = w->C[idx], av = w->A[idx];
        if (cv == 0 && (!need_d || av == 0)) continue;
        int r = idx / N, c = idx % N;
        if (r != c) {
            int u = r < c ? r : c, v = r < c ? c : r;
            long pp = pair_pos(N, u, v);
            if (!w->cmark[pp]) { w->cmark[pp] = 1; w->cand[w->ncand++] = pp; }
            if (!w->cmark[P + pp]) { w->cmark[P + pp] = 1; w->cand[w->ncand++] = P + pp; }
        } else {
            w->diag[w->ndiag++] = r;
            if (r < mindiag) mindiag = r;
        }
    }
    if (w->ndiag > 0) {
        for (int l = (mindiag > 1 ? mindiag : 1); l < N; l++) {
            long cc = 2 * P + (l - 1);
            if (!w->cmark[cc]) { w->cmark[cc] = 1; w->cand[w->ncand++] = cc; }
        }
    }
    /* expansion coefficients */
    long nout = 0;
    for (long t = 0; t < w->ncand; t++) {
        long c = w->cand[t];
        w->cmark[c] = 0;
        cplx trC = 0, trA = 0;
        if (c >= 2 * P) {
            int l = (int)(c - 2 * P) + 1;
            for (int q = 0; q < w->ndiag; q++) {
                int r = w->diag[q];
                double dv = dval(l, r);
                if (dv == 0.0) continue;
                int idx = r * N + r;
                trC += dv * w->C[idx];
                trA += dv * w->A[idx];
            }
        } else {
            int ne = basis_entries(N, c, w->fr, w->fc, w->fv);
            for (int q = 0; q < ne; q++) {
                /* Tr(F_c X) = sum_{(r,k)} (F_c)_{rk} X_{kr} */
                int idx = w->fc[q] * N + w->fr[q];
                if (!w->mark[idx]) continue;
                trC += w->fv[q] * w->C[idx];
                trA += w->fv[q] * w->A[idx];
            }
        }
        double fv = creal(-I * trC);
        double dv = need_d ? creal(trA) : 0.0;
        if (fabs(fv) < ZERO_TOL) fv = 0.0;
        if (fabs(dv) < ZERO_TOL) dv = 0.0;
        if (fv == 0.0 && dv == 0.0) continue;
        c_out[nout] = c;
        f_out[nout] = fv;
        d_out[nout] = dv;
        nout++;
    }
    ws_clear(w);
    return nout;
}

/* ------------------------------------------------------------------------ */
/* Structure-constant tables (Table 1, step 2.2)                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int N;
    long M;
    long* start;   /* M+1 offsets into the entry arrays, per first index a */
    int* b;        /* second index */
    int* c;        /* third index  */
    double* f;     /* f_abc        */
    double* d;     /* d_abc        */
} table_t;

/* Builds, for every first index a, the list of (b, c, f_abc, d_abc) with f or d nonzero. */
static table_t* table_build(int N) {
    long M = (long)N * N - 1;
    table_t* T = calloc(1, sizeof(table_t));
    T->N = N;
    T->M = M;
    T->start = calloc((size_t)M + 1, sizeof(long));
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    /* pass 1: counts */
    long* cnt = calloc((size_t)M, sizeof(long));
#pragma omp parallel num_threads(nth)
    {
        ws_t* w = ws_new(N);
        long* ol = malloc(sizeof(long) * (size_t)M);
        long* cb = malloc(sizeof(long) * (size_t)M);
        double* fb = malloc(sizeof(double) * (size_t)M);
        double* db = malloc(sizeof(double) * (size_t)M);
#pragma omp for schedule(dynamic, 16)
        for (long a = 0; a < M; a++) {
            long no = overlap_list(N, a, ol);
            long tot = 0;
            for (long t = 0; t < no; t++) tot += fiber(w, a, ol[t], 1, cb, fb, db);
            cnt[a] = tot;
        }
        free(ol); free(cb); free(fb); free(db);
        ws_free(w);
    }
    for (long a = 0; a < M; a++) T->start[a + 1] = T->start[a] + cnt[a];
    long total = T->start[M];
    T->b = malloc(sizeof(int) * (size_t)total);
    T->c = malloc(sizeof(int) * (size_t)total);
    T->f = malloc(sizeof(double) * (size_t)total);
    T->d = malloc(sizeof(double) * (size_t)total);
    /* pass 2: fill */
#pragma omp parallel num_threads(nth)
    {
        ws_t* w = ws_new(N);
        long* ol = malloc(sizeof(long) * (size_t)M);
        long* cb = malloc(sizeof(long) * (size_t)M);
        double* fb = malloc(sizeof(double) * (size_t)M);
        double* db = malloc(sizeof(double) * (size_t)M);
#pragma omp for schedule(dynamic, 16)
        for (long a = 0; a < M; a++) {
            long no = overlap_list(N, a, ol);
            long pos = T->start[a];
            for (long t = 0; t < no; t++) {
                long nf = fiber(w, a, ol[t], 1, cb, fb, db);
                for (long q = 0; q < nf; q++) {
                    T->b[pos] = (int)ol[t];
                    T->c[pos] = (int)cb[q];
                    T->f[pos] = fb[q];
                    T->d[pos] = db[q];
                    pos++;
                }
            }
        }
        free(ol); free(cb); free(fb); free(db);
        ws_free(w);
    }
    free(cnt);
    return T;
}

static void table_free(table_t* T) {
    free(T->start); free(T->b); free(T->c); free(T->f); free(T->d); free(T);
}

/* Counts of nonzero ordered f and d triples. */
void or_fd_count(int N, long* nf, long* nd) {
    table_t* T = table_build(N);
    long cf = 0, cd = 0;
    for (long e = 0; e < T->start[T->M]; e++) { if (T->f[e] != 0.0) cf++; if (T->d[e] != 0.0) cd++; }
    *nf = cf; *nd = cd;
    table_free(T);
}

/* All ordered (m, n, s) with f_mns (which=0) or d_mns (which=1) nonzero, m-major.
   Returns the count; writes min(count, cap) entries. */
long or_fd_enumerate(int N, int which, int32_t* mns, double* val, long cap) {
    table_t* T = table_build(N);
    long n = 0;
    for (long a = 0; a < T->M; a++) {
        for (long e = T->start[a]; e < T->start[a + 1]; e++) {
            double v = which == 0 ? T->f[e] : T->d[e];
            if (v == 0.0) continue;
            if (n < cap) {
                mns[3 * n] = (int32_t)a;
                mns[3 * n + 1] = T->b[e];
                mns[3 * n + 2] = T->c[e];
                val[n] = v;
            }
            n++;
        }
    }
    table_free(T);
    return n;
}

/* ------------------------------------------------------------------------ */
/* Expansion and reconstruction (Eqs. (6), (7); Table 1 steps 2.1, 2.6, 3.2)  */
/* ------------------------------------------------------------------------ */

/* a_j = Tr(F_j A) for j = 0..M-1 (complex; real when A is Hermitian). */
void or_expand(int N, const double* A /* N*N complex */, double* a /* M complex */) {
    long M = (long)N * N - 1;
    const cplx* Ac = (const cplx*)A;
    cplx* ac = (cplx*)a;
#pragma omp parallel
    {
        int* r = malloc(sizeof(int) * N);
        int* c = malloc(sizeof(int) * N);
        cplx* v = malloc(sizeof(cplx) * N);
#pragma omp for schedule(static)
        for (long j = 0; j < M; j++) {
            int n = basis_entries(N, j, r, c, v);
            cplx s = 0;
            for (int t = 0; t < n; t++) s += v[t] * Ac[(size_t)c[t] * N + r[t]];
            ac[j] = s;
        }
        free(r); free(c); free(v);
    }
}

/* rho = 1/N + sum_i v_i F_i (Eq. (7)) */
void or_reconstruct(int N, const double* v, double* rho /* N*N complex */) {
    long M = (long)N * N - 1;
    cplx* R = (cplx*)rho;
    for (size_t t = 0; t < (size_t)N * N; t++) R[t] = 0;
    for (int x = 0; x < N; x++) R[(size_t)x * N + x] = 1.0 / N;
    int* r = malloc(sizeof(int) * N);
    int* c = malloc(sizeof(int) * N);
    cplx* e = malloc(sizeof(cplx) * N);
    for (long i = 0; i < M; i++) {
        int n = basis_entries(N, i, r, c, e);
        for (int t = 0; t < n; t++) R[(size_t)r[t] * N + c[t]] += v[i] * e[t];
    }
    free(r); free(c); free(e);
}

/* ------------------------------------------------------------------------ */
/* Dense data preparation: Eqs. (13), (14), (15) (Table 1, steps 2.3-2.5)     */
/* ------------------------------------------------------------------------ */

/*
 * Rows `rows[0..nrows)` of Q = Q_H + Q_D and the full vector K, for a dense
 * Hermitian H (N x N) and a dense Kossakowski matrix gamma (M x M, complex,
 * in the basis order above). Qrows is nrows x M row-major.
 *
 *   q_sn  = sum_m h_m f_mns                                        (13)
 *   k_s   = (i/N) sum_mn gamma_mn f_mns                             (14)
 *   r_sn  = -1/4 sum_jkl gamma_jk (z_jln f_kls + conj(z_kln) f_jls)  (15)
 *
 * The sums run over the nonzero structure constants only (step 2.2): for
 * output row s, (k, l) runs over the nonzeros f_kls = f_skl (cyclic) and,
 * for each l, (j, n) over the nonzeros z_jln = f_lnj + i d_lnj.
 * maximag (optional) receives max |Im r_sn| seen (should be ~0).
 */
void or_prepare_dense(int N, const double* H, const double* gamma, const long* rows, long nrows,
                      double* Qrows, double* K, double* maximag) {
    long M = (long)N * N - 1;
    const cplx* G = (const cplx*)gamma;
    /* step 2.1: h */
    double* hc = malloc(sizeof(double) * 2 * (size_t)M);
    or_expand(N, H, hc);
    table_t* T = table_build(N);
    double mi = 0.0;
    /* step 2.4: K over all s */
    if (K) {
        for (long s = 0; s < M; s++) {
            cplx acc = 0;
            for (long e = T->start[s]; e < T->start[s + 1]; e++) {
                if (T->f[e] == 0.0) continue;
                long m = T->b[e], n = T->c[e];
                acc += G[(size_t)m * M + n] * T->f[e]; /* f_mns = f_smn */
            }
            K[s] = creal(I * acc / (double)N);
        }
    }
#pragma omp parallel reduction(max : mi)
    {
        cplx* row = malloc(sizeof(cplx) * (size_t)M);
#pragma omp for schedule(dynamic, 1)
        for (long t = 0; t < nrows; t++) {
            long s = rows[t];
            for (long n = 0; n < M; n++) row[n] = 0;
            /* Eq. (13): q_sn = sum_m h_m f_mns, with f_mns = f_smn */
            for (long e = T->start[s]; e < T->start[s + 1]; e++) {
                if (T->f[e] == 0.0) continue;
                long m = T->b[e], n = T->c[e];
                row[n] += hc[2 * m] * T->f[e];
            }
            /* Eq. (15), first term: sum_{k,l} f_kls sum_{j,n} gamma_jk z_jln */
            for (long e = T->start[s]; e < T->start[s + 1]; e++) {
                double fkls = T->f[e];
                if (fkls == 0.0) continue;
                long k = T->b[e], l = T->c[e];
                for (long q = T->start[l]; q < T->start[l + 1]; q++) {
                    long n = T->b[q], j = T->c[q];
                    cplx z = T->f[q] + I * T->d[q]; /* z_jln = f_lnj + i d_lnj */
                    row[n] += -0.25 * G[(size_t)j * M + k] * z * fkls;
                }
            }
            /* Eq. (15), second term: sum_{j,l} f_jls sum_{k,n} gamma_jk conj(z_kln) */
            for (long e = T->start[s]; e < T->start[s + 1]; e++) {
                double fjls = T->f[e];
                if (fjls == 0.0) continue;
                long j = T->b[e], l = T->c[e];
                for (long q = T->start[l]; q < T->start[l + 1]; q++) {
                    long n = T->b[q], k = T->c[q];
                    cplx zc = T->f[q] - I * T->d[q]; /* conj(z_kln) */
                    row[n] += -0.25 * G[(size_t)j * M + k] * zc * fjls;
                }
            }
            for (long n = 0; n < M; n++) {
                Qrows[(size_t)t * M + n] = creal(row[n]);
                double im = fabs(cimag(row[n]));
                if (im > mi) mi = im;
            }
        }
        free(row);
    }
    if (maximag) *maximag = mi;
    table_free(T);
    free(hc);
}

/* ------------------------------------------------------------------------ */
/* Factored Kossakowski matrix: gamma = sum_p g_p l_p l_p^dagger (Sec. 2)     */
/* ------------------------------------------------------------------------ */

/*
 * Jump operators L_p (N x N, complex) with rates g_p: l_p,j = Tr(F_j L_p0)
 * where L_p0 = L_p - c_p 1 and c_p = Tr(L_p)/N. The identity parts are moved
 * into the Hamiltonian: H_eff = H + sum_p (i g_p / 2)(conj(c_p) L_p0 - c_p L_p0^dagger).
 * Outputs: Heff (N x N complex), l (P x M complex).
 */
void or_jump_setup(int N, const double* H, int P, const double* rates, const double* Ls,
                   double* Heff, double* l) {
    size_t NN = (size_t)N * N;
    long M = (long)N * N - 1;
    const cplx* Hc = (const cplx*)H;
    cplx* He = (cplx*)Heff;
    for (size_t t = 0; t < NN; t++) He[t] = Hc[t];
    cplx* L0 = malloc(sizeof(cplx) * NN);
    for (int p = 0; p < P; p++) {
        const cplx* Lp = (const cplx*)(Ls + 2 * NN * p);
        cplx tr = 0;
        for (int x = 0; x < N; x++) tr += Lp[(size_t)x * N + x];
        cplx c = tr / (double)N;
        for (size_t t = 0; t < NN; t++) L0[t] = Lp[t];
        for (int x = 0; x < N; x++) L0[(size_t)x * N + x] -= c;
        double g = rates[p];
        for (int a = 0; a < N; a++)
            for (int b = 0; b < N; b++) {
                cplx l0ab = L0[(size_t)a * N + b];
                cplx l0dag_ab = conj(L0[(size_t)b * N + a]);
                He[(size_t)a * N + b] += (I * g / 2.0) * (conj(c) * l0ab - c * l0dag_ab);
            }
        or_expand(N, (const double*)L0, l + 2 * (size_t)M * p);
    }
    free(L0);
}

/*
 * Rows of Q and the full K for a Hamiltonian H (already including any
 * jump-operator trace shifts) and gamma = sum_p g_p l_p l_p^dagger with
 * sparse l_p. Structure constants are computed on the fly, only where a
 * nonzero of h or l_p makes them needed (step 2.2).
 *   Eq. (13): q_sn = sum_m h_m f_smn over h_m != 0.
 *   Eq. (14): k_s = (i/N) sum_p g_p sum_mn l_m conj(l_n) f_smn.
 *   Eq. (15): r_sn = -1/4 sum_p g_p sum_jkl l_j conj(l_k)(z_jln f_kls + conj(z_kln) f_jls).
 * Krows receives k_s for the requested rows only.
 */
void or_prepare_factored(int N, const double* H, int P, const double* rates, const double* l,
                         const long* rows, long nrows, double* Qrows, double* Krows) {
    long M = (long)N * N - 1;
    double* hc = malloc(sizeof(double) * 2 * (size_t)M);
    or_expand(N, H, hc);
    /* nonzero index lists */
    long nh = 0;
    long* hidx = malloc(sizeof(long) * (size_t)M);
    for (long m = 0; m < M; m++) if (hc[2 * m] != 0.0) hidx[nh++] = m;
    long* lcnt = calloc(P, sizeof(long));
    long** lidx = malloc(sizeof(long*) * P);
    for (int p = 0; p < P; p++) {
        const cplx* lp = (const cplx*)(l + 2 * (size_t)M * p);
        lidx[p] = malloc(sizeof(long) * (size_t)M);
        for (long m = 0; m < M; m++) if (lp[m] != 0) lidx[p][lcnt[p]++] = m;
    }
#pragma omp parallel
    {
        ws_t* w = ws_new(N);
        cplx* row = malloc(sizeof(cplx) * (size_t)M);
        long* c1 = malloc(sizeof(long) * (size_t)M);
        double* f1 = malloc(sizeof(double) * (size_t)M);
        double* d1 = malloc(sizeof(double) * (size_t)M);
        long* c2 = malloc(sizeof(long) * (size_t)M);
        double* f2 = malloc(sizeof(double) * (size_t)M);
        double* d2 = malloc(sizeof(double) * (size_t)M);
#pragma omp for schedule(dynamic, 1)
        for (long t = 0; t < nrows; t++) {
            long s = rows[t];
            for (long n = 0; n < M; n++) row[n] = 0;
            cplx kacc = 0;
            /* Eq. (13) */
            for (long q = 0; q < nh; q++) {
                long m = hidx[q];
                if (!overlap(N, s, m)) continue;
                long nf = fiber(w, s, m, 0, c1, f1, d1);
                for (long e = 0; e < nf; e++) row[c1[e]] += hc[2 * m] * f1[e];
            }
            for (int p = 0; p < P; p++) {
                const cplx* lp = (const cplx*)(l + 2 * (size_t)M * p);
                double g = rates[p];
                /* Eq. (14) */
                for (long q = 0; q < lcnt[p]; q++) {
                    long m = lidx[p][q];
                    if (!overlap(N, s, m)) continue;
                    long nf = fiber(w, s, m, 0, c1, f1, d1); /* (n, f_smn) */
                    for (long e = 0; e < nf; e++) {
                        long n = c1[e];
                        if (lp[n] == 0) continue;
                        kacc += g * lp[m] * conj(lp[n]) * f1[e];
                    }
                }
                /* Eq. (15), both terms: outer index x with l_x != 0 and f_{x l s} = f_{s x l} */
                for (long q = 0; q < lcnt[p]; q++) {
                    long x = lidx[p][q];
                    if (!overlap(N, s, x)) continue;
                    long nf = fiber(w, s, x, 0, c1, f1, d1); /* (l, f_sxl) */
                    for (long e = 0; e < nf; e++) {
                        long li = c1[e];
                        double fxls = f1[e];
                        for (long q2 = 0; q2 < lcnt[p]; q2++) {
                            long y = lidx[p][q2];
                            if (!overlap(N, y, li)) continue;
                            long nz = fiber(w, y, li, 1, c2, f2, d2); /* (n, f_yln, d_yln) */
                            for (long e2 = 0; e2 < nz; e2++) {
                                long n = c2[e2];
                                cplx z = f2[e2] + I * d2[e2];
                                /* term 1: k = x, j = y: l_j conj(l_k) z_jln f_kls */
                                row[n] += -0.25 * g * lp[y] * conj(lp[x]) * z * fxls;
                                /* term 2: j = x, k = y: l_j conj(l_k) conj(z_kln) f_jls */
                                row[n] += -0.25 * g * lp[x] * conj(lp[y]) * conj(z) * fxls;
                            }
                        }
                    }
                }
            }
            for (long n = 0; n < M; n++) Qrows[(size_t)t * M + n] = creal(row[n]);
            if (Krows) Krows[t] = creal(I * kacc / (double)N);
        }
        free(row); free(c1); free(f1); free(d1); free(c2); free(f2); free(d2);
        ws_free(w);
    }
    for (int p = 0; p < P; p++) free(lidx[p]);
    free(lidx); free(lcnt); free(hidx); free(hc);
}

/* ------------------------------------------------------------------------ */
/* RK4 integration of dv/dt = Q v + K (Eq. (10); Table 1, step 3.1)          */
/* ------------------------------------------------------------------------ */

static void matvec_dense(long M, const double* Q, const double* K, const double* x, double* y, int B) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < M; i++) {
        const double* qi = Q + (size_t)i * M;
        for (int b = 0; b < B; b++) {
            const double* xb = x + (size_t)b * M;
            double acc = K[i];
            for (long j = 0; j < M; j++) acc += qi[j] * xb[j];
            y[(size_t)b * M + i] = acc;
        }
    }
}

static void matvec_csr(long M, const int64_t* rowptr, const int64_t* col, const double* val,
                       const double* K, const double* x, double* y, int B) {
#pragma omp parallel for schedule(dynamic, 256)
    for (long i = 0; i < M; i++) {
        for (int b = 0; b < B; b++) {
            const double* xb = x + (size_t)b * M;
            double acc = K[i];
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) acc += val[e] * xb[col[e]];
            y[(size_t)b * M + i] = acc;
        }
    }
}

/* Classic fourth-order Runge-Kutta, weights 1/6, 1/3, 1/3, 1/6; V is B x M, updated in place. */
static void rk4_generic(long M, int B, double dt, long steps, double* V,
                        void (*mv)(const void*, const double*, double*), const void* ctx) {
    size_t n = (size_t)M * B;
    double* k1 = malloc(sizeof(double) * n);
    double* k2 = malloc(sizeof(double) * n);
    double* k3 = malloc(sizeof(double) * n);
    double* k4 = malloc(sizeof(double) * n);
    double* x = malloc(sizeof(double) * n);
    for (long st = 0; st < steps; st++) {
        mv(ctx, V, k1);
        for (size_t t = 0; t < n; t++) x[t] = V[t] + 0.5 * dt * k1[t];
        mv(ctx, x, k2);
        for (size_t t = 0; t < n; t++) x[t] = V[t] + 0.5 * dt * k2[t];
        mv(ctx, x, k3);
        for (size_t t = 0; t < n; t++) x[t] = V[t] + dt * k3[t];
        mv(ctx, x, k4);
        for (size_t t = 0; t < n; t++) V[t] += dt / 6.0 * (k1[t] + 2.0 * k2[t] + 2.0 * k3[t] + k4[t]);
    }
    free(k1); free(k2); free(k3); free(k4); free(x);
}

typedef struct { long M; const double* Q; const double* K; int B; } dense_ctx;
typedef struct { long M; const int64_t* rp; const int64_t* ci; const double* v; const double* K; int B; } csr_ctx;

static void mv_dense(const void* c, const double* x, double* y) {
    const dense_ctx* d = c;
    matvec_dense(d->M, d->Q, d->K, x, y, d->B);
}
static void mv_csr(const void* c, const double* x, double* y) {
    const csr_ctx* d = c;
    matvec_csr(d->M, d->rp, d->ci, d->v, d->K, x, y, d->B);
}

void or_rk4_dense(long M, const double* Q, const double* K, double* V, int B, double dt, long steps) {
    dense_ctx c = {M, Q, K, B};
    rk4_generic(M, B, dt, steps, V, mv_dense, &c);
}

void or_rk4_csr(long M, const int64_t* rowptr, const int64_t* col, const double* val, const double* K,
                double* V, int B, double dt, long steps) {
    csr_ctx c = {M, rowptr, col, val, K, B};
    rk4_generic(M, B, dt, steps, V, mv_csr, &c);
}

/* ------------------------------------------------------------------------ */
/* Periodically driven dimer (Sec. 3, Eq. (16)): H(t) = H0 + eps(t) H1 with   */
/* the square wave eps(t) = E + A Theta(t), Theta = +1 for 0 <= t < T/2 and   */
/* -1 for T/2 <= t < T, period T. Q_H is linear in H and K does not involve H */
/* (L(1) has no Hamiltonian part), so the ODE of Eq. (10) becomes             */
/*     dv/dt = (Q0 + eps(t) Q1) v + K,                                        */
/* Q0 from (H0, dissipator), Q1 = Q_H of H1 alone. Classic RK4 evaluates eps  */
/* at the stage times t_k, t_k + dt/2, t_k + dt (t_k = t0 + k dt) as seen from */
/* inside the step: the first two from the right, the last as the limit from */
/* the left, so a step that ends on a switch integrates one constant system.  */
/* ------------------------------------------------------------------------ */

double or_drive(double t, double E, double A, double T) {
    double r = fmod(t, T);
    if (r < 0) r += T;
    return r < 0.5 * T ? E + A : E - A;
}

/* The limit from the left, eps(t-): at a switch time it is the value of the   */
/* half period that ends there.                                               */
double or_drive_left(double t, double E, double A, double T) {
    double r = fmod(t, T);
    if (r <= 0) r += T;
    return r <= 0.5 * T ? E + A : E - A;
}

/* t0 + (k + c) dt, c in {0, 1/2, 1}: one product and one sum */
static double stage_time(double t0, long k, double c, double dt) {
    const double kc = (double)k + c;
    volatile double p = kc * dt; /* rounded on its own, never fused with the sum */
    return t0 + p;
}

/* y = (Q0 + e Q1) x + K for dense M x M Q0, Q1; B states */
static void matvec_drive(long M, const double* Q0, const double* Q1, double e, const double* K, const double* x,
                         double* y, int B) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < M; i++) {
        const double* q0 = Q0 + (size_t)i * M;
        const double* q1 = Q1 + (size_t)i * M;
        for (int b = 0; b < B; b++) {
            const double* xb = x + (size_t)b * M;
            double a0 = K[i], a1 = 0.0;
            for (long j = 0; j < M; j++) {
                a0 += q0[j] * xb[j];
                a1 += q1[j] * xb[j];
            }
            y[(size_t)b * M + i] = a0 + e * a1;
        }
    }
}

void or_rk4_drive(long M, const double* Q0, const double* Q1, const double* K, double* V, int B, double dt,
                  long steps, double t0, double E, double A, double T) {
    size_t n = (size_t)M * B;
    double* k1 = malloc(sizeof(double) * n);
    double* k2 = malloc(sizeof(double) * n);
    double* k3 = malloc(sizeof(double) * n);
    double* k4 = malloc(sizeof(double) * n);
    double* x = malloc(sizeof(double) * n);
    for (long st = 0; st < steps; st++) {
        const double e1 = or_drive(stage_time(t0, st, 0.0, dt), E, A, T);
        const double e2 = or_drive(stage_time(t0, st, 0.5, dt), E, A, T);
        const double e4 = or_drive_left(stage_time(t0, st, 1.0, dt), E, A, T);
        matvec_drive(M, Q0, Q1, e1, K, V, k1, B);
        for (size_t t = 0; t < n; t++) x[t] = V[t] + 0.5 * dt * k1[t];
        matvec_drive(M, Q0, Q1, e2, K, x, k2, B);
        for (size_t t = 0; t < n; t++) x[t] = V[t] + 0.5 * dt * k2[t];
        matvec_drive(M, Q0, Q1, e2, K, x, k3, B);
        for (size_t t = 0; t < n; t++) x[t] = V[t] + dt * k3[t];
        matvec_drive(M, Q0, Q1, e4, K, x, k4, B);
        for (size_t t = 0; t < n; t++) V[t] += dt / 6.0 * (k1[t] + 2.0 * k2[t] + 2.0 * k3[t] + k4[t]);
    }
    free(k1); free(k2); free(k3); free(k4); free(x);
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
