/*
 * Precision-generic body of the CPU oracle.  Included twice by lhaf_oracle.c,
 * once with REAL = double and once with REAL = long double.  TEST
 * INFRASTRUCTURE ONLY: nothing in the product library links this file.
 *
 * Required macros on inclusion:
 *   SFX(name)  symbol suffixing, e.g. name##_d
 *   REAL       real type, CPLX the matching C99 complex type
 *   RSQRT(x)   real square root, RABS(x) real |x|, ZABS(z) complex |z|
 *   ZCONJ(z), ZRE(z), ZIM(z)
 *
 * What is computed (all definitions are from Quesada et al., "Quadratic speedup
 * for simulating Gaussian boson sampling", cited here as "the paper"):
 *   lhaf(A) = sum over single-pair matchings (every vertex is either covered by a
 *   loop, weight A_ii, or paired with one other vertex, weight A_ij) of the
 *   product of weights -- Sec. II, the definition given after Eq. (11), the
 *   loop-hafnian analogue of the hafnian of Eq. (6).
 *
 * Two independent evaluators:
 *   dp   : the definition, memoised over vertex subsets (lowest remaining vertex
 *          is either a loop or paired with some j).  O(2^N N).
 *   pt   : the power-trace subset sum the paper benchmarks in Sec. IV (the
 *          algorithm of its Ref. [bjorklund2018faster]), with characteristic
 *          polynomials by La Budde's method (Sec. IV, Ref. [rehman2011budde])
 *          and power traces by Newton's identities.  Steps, per pair subset S:
 *            1. C = X_S A0_S (A0 = A with zero diagonal, X_S swaps pair halves)
 *            2. Householder reduction of C to upper Hessenberg form H
 *            3. La Budde recurrence for det(xI - H)
 *            4. Newton's identities -> p_k = tr(C^k), k = 1..n
 *            5. loop terms q_k = d_S^T C^(k-1) (X_S d_S) by dense mat-vecs on C
 *            6. c_k = p_k/(2k) + q_k/2, e = exp(sum c_k eta^k) coefficients
 *            7. term = (-1)^(n-|S|) e_n, summed with Neumaier compensation
 *          Odd N is padded with one vertex of loop weight 1 and no edges,
 *          which leaves the value unchanged.
 */

/* ---------------------------------------------------------------------- */
/* brute force over single-pair matchings (definition)                    */
/* ---------------------------------------------------------------------- */
int SFX(oracle_lhaf_dp)(const double *A, int N, REAL *out)
{
    if (N < 0 || N > ORACLE_DP_MAX_N || !out || (N > 0 && !A)) return -1;
    if (N == 0) { out[0] = 1; out[1] = 0; return 0; }
    size_t size = (size_t)1 << N;
    CPLX *f = (CPLX *)malloc(size * sizeof(CPLX));
    if (!f) return -2;
    f[0] = 1;
    for (size_t mask = 1; mask < size; ++mask) {
        int i = __builtin_ctzll((unsigned long long)mask);
        size_t rest = mask & ~((size_t)1 << i);
        CPLX aii = (REAL)A[2 * (i * N + i)] + (REAL)A[2 * (i * N + i) + 1] * I;
        CPLX tot = aii * f[rest];
        size_t r = rest;
        while (r) {
            int j = __builtin_ctzll((unsigned long long)r);
            CPLX aij = (REAL)A[2 * (i * N + j)] + (REAL)A[2 * (i * N + j) + 1] * I;
            tot += aij * f[rest & ~((size_t)1 << j)];
            r &= r - 1;
        }
        f[mask] = tot;
    }
    out[0] = ZRE(f[size - 1]);
    out[1] = ZIM(f[size - 1]);
    free(f);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* dense linear algebra on small complex matrices (row-major, m x m)      */
/* ---------------------------------------------------------------------- */

/* Householder reduction to upper Hessenberg form, in place (Golub & Van Loan,
 * Matrix Computations, Alg. 7.4.2, complex reflectors P = I - 2 v v^H / v^H v). */
static void SFX(hessenberg)(CPLX *H, int m, CPLX *v)
{
    for (int k = 0; k + 2 < m; ++k) {
        REAL xnorm2 = 0;
        for (int r = k + 1; r < m; ++r) {
            REAL a = ZABS(H[r * m + k]);
            xnorm2 += a * a;
        }
        if (xnorm2 == 0) continue;
        REAL xnorm = RSQRT(xnorm2);
        CPLX x0 = H[(k + 1) * m + k];
        REAL ax0 = ZABS(x0);
        CPLX phase = ax0 == 0 ? (CPLX)1 : x0 / ax0;
        for (int r = k + 1; r < m; ++r) v[r] = H[r * m + k];
        v[k + 1] = x0 + phase * xnorm;
        REAL vnorm2 = 0;
        for (int r = k + 1; r < m; ++r) {
            REAL a = ZABS(v[r]);
            vnorm2 += a * a;
        }
        if (vnorm2 == 0) continue;
        REAL two_over = 2 / vnorm2;
        /* left: H[k+1:, k:] -= (2/v^H v) v (v^H H[k+1:, k:]) */
        for (int c = k; c < m; ++c) {
            CPLX w = 0;
            for (int r = k + 1; r < m; ++r) w += ZCONJ(v[r]) * H[r * m + c];
            w *= two_over;
            for (int r = k + 1; r < m; ++r) H[r * m + c] -= v[r] * w;
        }
        /* right: H[:, k+1:] -= (2/v^H v) (H[:, k+1:] v) v^H */
        for (int r = 0; r < m; ++r) {
            CPLX u = 0;
            for (int c = k + 1; c < m; ++c) u += H[r * m + c] * v[c];
            u *= two_over;
            for (int c = k + 1; c < m; ++c) H[r * m + c] -= u * ZCONJ(v[c]);
        }
        /* the reduced column is exactly -phase*||x|| e_1 */
        H[(k + 1) * m + k] = -phase * xnorm;
        for (int r = k + 2; r < m; ++r) H[r * m + k] = 0;
    }
}

/* La Budde's recurrence (Rehman & Ipsen, 2011) for the characteristic
 * polynomials of the leading principal submatrices of an upper Hessenberg H.
 * With 1-based indices, p_0 = 1 and
 *   p_i(x) = (x - h_ii) p_{i-1}(x)
 *            - sum_{k=1}^{i-1} h_{i-k,i} (prod_{j=i-k+1}^{i} h_{j,j-1}) p_{i-k-1}(x).
 * poly is (m+1) x (m+1): poly[i*(m+1) + t] = coefficient of x^t in p_i.
 * On return coef[t] = coefficient of x^t of det(xI - H), t = 0..m. */
static void SFX(labudde)(const CPLX *H, int m, CPLX *poly, CPLX *coef)
{
    int W = m + 1;
    for (int i = 0; i < W * W; ++i) poly[i] = 0;
    poly[0] = 1;
#define HH(a, b) H[((a) - 1) * m + ((b) - 1)] /* 1-based accessor */
    for (int i = 1; i <= m; ++i) {
        CPLX *pi = poly + i * W;
        const CPLX *pim1 = poly + (i - 1) * W;
        for (int t = 0; t <= i; ++t) {
            CPLX acc = 0;
            if (t >= 1) acc += pim1[t - 1];
            if (t <= i - 1) acc -= HH(i, i) * pim1[t];
            pi[t] = acc;
        }
        CPLX prod = 1;
        for (int k = 1; k <= i - 1; ++k) {
            prod *= HH(i - k + 1, i - k);
            CPLX beta = HH(i - k, i) * prod;
            const CPLX *pq = poly + (i - k - 1) * W;
            for (int t = 0; t <= i - k - 1; ++t) pi[t] -= beta * pq[t];
        }
    }
#undef HH
    for (int t = 0; t <= m; ++t) coef[t] = poly[m * W + t];
}

/* Newton's identities: power sums p_k = tr(M^k), k = 1..K, from the monic
 * characteristic polynomial x^m + a_1 x^(m-1) + ... + a_m (a_j = 0 for j > m,
 * which continues the sequence by the Cayley-Hamilton recurrence):
 *   p_k = -k a_k - sum_{j=1}^{k-1} a_j p_{k-j}. */
static void SFX(newton)(const CPLX *coef, int m, int K, CPLX *p /* K+1 */)
{
    p[0] = m;
    for (int k = 1; k <= K; ++k) {
        CPLX ak = k <= m ? coef[m - k] : (CPLX)0;
        CPLX acc = -(REAL)k * ak;
        for (int j = 1; j <= k - 1 && j <= m; ++j) acc -= coef[m - j] * p[k - j];
        p[k] = acc;
    }
}

/* workspace for one subset term */
typedef struct {
    CPLX *C, *H, *v, *poly, *coef, *p, *q, *w, *w2, *c, *e, *dS, *zS;
} SFX(ws_t);

static int SFX(ws_alloc)(SFX(ws_t) *ws, int N)
{
    int M = N + 2;
    ws->C = (CPLX *)calloc((size_t)M * M, sizeof(CPLX));
    ws->H = (CPLX *)calloc((size_t)M * M, sizeof(CPLX));
    ws->poly = (CPLX *)calloc((size_t)(M + 1) * (M + 1), sizeof(CPLX));
    ws->v = (CPLX *)calloc(M, sizeof(CPLX));
    ws->coef = (CPLX *)calloc(M + 1, sizeof(CPLX));
    ws->p = (CPLX *)calloc(M + 1, sizeof(CPLX));
    ws->q = (CPLX *)calloc(M + 1, sizeof(CPLX));
    ws->w = (CPLX *)calloc(M, sizeof(CPLX));
    ws->w2 = (CPLX *)calloc(M, sizeof(CPLX));
    ws->c = (CPLX *)calloc(M + 1, sizeof(CPLX));
    ws->e = (CPLX *)calloc(M + 1, sizeof(CPLX));
    ws->dS = (CPLX *)calloc(M, sizeof(CPLX));
    ws->zS = (CPLX *)calloc(M, sizeof(CPLX));
    return (ws->C && ws->H && ws->poly && ws->v && ws->coef && ws->p && ws->q && ws->w &&
            ws->w2 && ws->c && ws->e && ws->dS && ws->zS) ? 0 : -2;
}

static void SFX(ws_free)(SFX(ws_t) *ws)
{
    free(ws->C); free(ws->H); free(ws->poly); free(ws->v); free(ws->coef); free(ws->p);
    free(ws->q); free(ws->w); free(ws->w2); free(ws->c); free(ws->e); free(ws->dS); free(ws->zS);
}

/* The padded, even-dimension matrix the subset sum runs on: Ap (Np x Np). */
static CPLX *SFX(padded)(const double *A, int N, int *Np_out)
{
    int Np = N + (N & 1);
    CPLX *Ap = (CPLX *)calloc((size_t)Np * Np + 1, sizeof(CPLX));
    if (!Ap) return NULL;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            Ap[i * Np + j] = (REAL)A[2 * (i * N + j)] + (REAL)A[2 * (i * N + j) + 1] * I;
    if (Np != N) Ap[N * Np + N] = 1; /* extra vertex: loop weight 1, no edges */
    *Np_out = Np;
    return Ap;
}

/* One signed subset term (-1)^(n-|S|) [eta^n] exp(sum_k c_k eta^k). */
static CPLX SFX(subset_term)(const CPLX *Ap, int Np, unsigned long long mask, SFX(ws_t) *ws)
{
    int n = Np / 2;
    int s = __builtin_popcountll(mask);
    int m = 2 * s;
    int idx[128];
    int t = 0;
    for (int i = 0; i < n; ++i)
        if (mask >> i & 1ULL) idx[t++] = i;
    for (int i = 0; i < s; ++i) idx[s + i] = idx[i] + n;
    /* step 1: C = X_S A0_S; row r of C is row X(r) of A0_S, X swaps halves */
    for (int r = 0; r < m; ++r) {
        int xr = r < s ? r + s : r - s;
        for (int c = 0; c < m; ++c) {
            int a = idx[xr], b = idx[c];
            ws->C[r * m + c] = (a == b) ? (CPLX)0 : Ap[a * Np + b];
        }
        ws->dS[r] = Ap[idx[r] * Np + idx[r]];
        ws->zS[r] = Ap[idx[xr] * Np + idx[xr]];
    }
    /* steps 2-4: power traces p_k = tr(C^k) */
    if (m > 0) {
        for (int i = 0; i < m * m; ++i) ws->H[i] = ws->C[i];
        SFX(hessenberg)(ws->H, m, ws->v);
        SFX(labudde)(ws->H, m, ws->poly, ws->coef);
        SFX(newton)(ws->coef, m, n, ws->p);
    } else {
        for (int k = 0; k <= n; ++k) ws->p[k] = 0;
    }
    /* step 5: loop terms q_k = d_S^T C^(k-1) z_S by repeated mat-vecs */
    for (int r = 0; r < m; ++r) ws->w[r] = ws->zS[r];
    for (int k = 1; k <= n; ++k) {
        CPLX acc = 0;
        for (int r = 0; r < m; ++r) acc += ws->dS[r] * ws->w[r];
        ws->q[k] = acc;
        if (k == n) break;
        for (int r = 0; r < m; ++r) {
            CPLX u = 0;
            for (int c = 0; c < m; ++c) u += ws->C[r * m + c] * ws->w[c];
            ws->w2[r] = u;
        }
        for (int r = 0; r < m; ++r) ws->w[r] = ws->w2[r];
    }
    /* step 6: c_k and the coefficients of exp(sum_k c_k eta^k):
     * e_0 = 1, e_k = (1/k) sum_{j=1}^{k} j c_j e_{k-j}. */
    for (int k = 1; k <= n; ++k) ws->c[k] = ws->p[k] / (REAL)(2 * k) + ws->q[k] / (REAL)2;
    ws->e[0] = 1;
    for (int k = 1; k <= n; ++k) {
        CPLX acc = 0;
        for (int j = 1; j <= k; ++j) acc += (REAL)j * ws->c[j] * ws->e[k - j];
        ws->e[k] = acc / (REAL)k;
    }
    /* step 7: sign (-1)^(n - |S|) */
    return ((n - s) & 1) ? -ws->e[n] : ws->e[n];
}

/* Neumaier (Kahan-Babuska) accumulation of one real stream */
static inline void SFX(neumaier)(REAL *sum, REAL *comp, REAL x)
{
    REAL t = *sum + x;
    if (RABS(*sum) >= RABS(x)) *comp += (*sum - t) + x;
    else *comp += (x - t) + *sum;
    *sum = t;
}

int SFX(oracle_term)(const double *A, int N, unsigned long long mask, REAL *out)
{
    if (N < 1 || N > ORACLE_PT_MAX_N || !A || !out) return -1;
    int Np;
    CPLX *Ap = SFX(padded)(A, N, &Np);
    if (!Ap) return -2;
    int n = Np / 2;
    if (n < 64 && (mask >> n) != 0) { free(Ap); return -1; }
    SFX(ws_t) ws;
    if (SFX(ws_alloc)(&ws, Np)) { SFX(ws_free)(&ws); free(Ap); return -2; }
    CPLX t = SFX(subset_term)(Ap, Np, mask, &ws);
    out[0] = ZRE(t);
    out[1] = ZIM(t);
    SFX(ws_free)(&ws);
    free(Ap);
    return 0;
}

/* Signed terms for a list of subset masks (each computed exactly as in
 * oracle_term), spread over threads; out receives 2 * count reals. */
int SFX(oracle_terms)(const double *A, int N, const unsigned long long *masks, long long count, int nthreads,
                      REAL *out)
{
    if (N < 1 || N > ORACLE_PT_MAX_N || !A || !out || count < 0 || (count > 0 && !masks)) return -1;
    int Np;
    CPLX *Ap = SFX(padded)(A, N, &Np);
    if (!Ap) return -2;
    int n = Np / 2;
    for (long long j = 0; j < count; ++j)
        if (n < 64 && (masks[j] >> n) != 0) { free(Ap); return -1; }
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        SFX(ws_t) ws;
        int bad = SFX(ws_alloc)(&ws, Np);
        if (bad) {
#pragma omp atomic write
            err = bad;
        }
#pragma omp for schedule(dynamic, 16)
        for (long long j = 0; j < count; ++j) {
            if (bad) continue;
            CPLX t = SFX(subset_term)(Ap, Np, masks[j], &ws);
            out[2 * j] = ZRE(t);
            out[2 * j + 1] = ZIM(t);
        }
        SFX(ws_free)(&ws);
    }
    free(Ap);
    return err;
}

/* Whole loop hafnian by the subset sum.  Subsets are visited in mask order in
 * fixed chunks of ORACLE_CHUNK masks; each chunk is summed in order with
 * Neumaier compensation and the chunk results are combined in chunk order, so
 * the result does not depend on the number of threads. */
int SFX(oracle_lhaf_pt)(const double *A, int N, int nthreads, REAL *out, REAL *abs_sum)
{
    if (N < 0 || N > ORACLE_PT_MAX_N || !out || (N > 0 && !A)) return -1;
    if (N == 0) {
        out[0] = 1; out[1] = 0;
        if (abs_sum) *abs_sum = 1;
        return 0;
    }
    int Np;
    CPLX *Ap = SFX(padded)(A, N, &Np);
    if (!Ap) return -2;
    int n = Np / 2;
    unsigned long long total = 1ULL << n;
    unsigned long long nchunks = (total + ORACLE_CHUNK - 1) / ORACLE_CHUNK;
    REAL *part = (REAL *)calloc(nchunks * 5, sizeof(REAL));
    if (!part) { free(Ap); return -2; }
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        SFX(ws_t) ws;
        int bad = SFX(ws_alloc)(&ws, Np);
        if (bad) {
#pragma omp atomic write
            err = bad;
        }
#pragma omp for schedule(dynamic, 1)
        for (long long ch = 0; ch < (long long)nchunks; ++ch) {
            if (bad) continue;
            REAL sr = 0, cr = 0, si = 0, ci = 0, ab = 0;
            unsigned long long lo = (unsigned long long)ch * ORACLE_CHUNK;
            unsigned long long hi = lo + ORACLE_CHUNK < total ? lo + ORACLE_CHUNK : total;
            for (unsigned long long mask = lo; mask < hi; ++mask) {
                CPLX t = SFX(subset_term)(Ap, Np, mask, &ws);
                SFX(neumaier)(&sr, &cr, ZRE(t));
                SFX(neumaier)(&si, &ci, ZIM(t));
                ab += ZABS(t);
            }
            part[5 * ch + 0] = sr; part[5 * ch + 1] = cr;
            part[5 * ch + 2] = si; part[5 * ch + 3] = ci;
            part[5 * ch + 4] = ab;
        }
        SFX(ws_free)(&ws);
    }
    if (err) { free(part); free(Ap); return err; }
    REAL sr = 0, cr = 0, si = 0, ci = 0, ab = 0;
    for (unsigned long long ch = 0; ch < nchunks; ++ch) {
        SFX(neumaier)(&sr, &cr, part[5 * ch + 0]);
        SFX(neumaier)(&sr, &cr, part[5 * ch + 1]);
        SFX(neumaier)(&si, &ci, part[5 * ch + 2]);
        SFX(neumaier)(&si, &ci, part[5 * ch + 3]);
        ab += part[5 * ch + 4];
    }
    out[0] = sr + cr;
    out[1] = si + ci;
    if (abs_sum) *abs_sum = ab;
    free(part);
    free(Ap);
    return 0;
}

/* Characteristic polynomial coefficients of a general m x m matrix, through
 * Householder Hessenberg reduction and La Budde: coef[2t], coef[2t+1] = re, im
 * of the coefficient of x^t in det(xI - M), t = 0..m. */
int SFX(oracle_charpoly)(const double *Min, int m, REAL *coef)
{
    if (m < 0 || m > 128 || !coef || (m > 0 && !Min)) return -1;
    CPLX *H = (CPLX *)calloc((size_t)m * m + 1, sizeof(CPLX));
    CPLX *v = (CPLX *)calloc(m + 1, sizeof(CPLX));
    CPLX *poly = (CPLX *)calloc((size_t)(m + 1) * (m + 1), sizeof(CPLX));
    CPLX *cf = (CPLX *)calloc(m + 1, sizeof(CPLX));
    if (!H || !v || !poly || !cf) { free(H); free(v); free(poly); free(cf); return -2; }
    for (int i = 0; i < m * m; ++i) H[i] = (REAL)Min[2 * i] + (REAL)Min[2 * i + 1] * I;
    SFX(hessenberg)(H, m, v);
    SFX(labudde)(H, m, poly, cf);
    if (m == 0) cf[0] = 1;
    for (int t = 0; t <= m; ++t) { coef[2 * t] = ZRE(cf[t]); coef[2 * t + 1] = ZIM(cf[t]); }
    free(H); free(v); free(poly); free(cf);
    return 0;
}

/* Power traces tr(M^k), k = 1..K, by Hessenberg + La Budde + Newton. */
int SFX(oracle_power_traces)(const double *Min, int m, int K, REAL *p)
{
    if (m < 1 || m > 128 || K < 1 || !Min || !p) return -1;
    REAL *cf = (REAL *)calloc(2 * (m + 1), sizeof(REAL));
    CPLX *coef = (CPLX *)calloc(m + 1, sizeof(CPLX));
    CPLX *pk = (CPLX *)calloc(K + 1, sizeof(CPLX));
    if (!cf || !coef || !pk) { free(cf); free(coef); free(pk); return -2; }
    int rc = SFX(oracle_charpoly)(Min, m, cf);
    if (rc == 0) {
        for (int t = 0; t <= m; ++t) coef[t] = cf[2 * t] + cf[2 * t + 1] * I;
        SFX(newton)(coef, m, K, pk);
        for (int k = 1; k <= K; ++k) { p[2 * (k - 1)] = ZRE(pk[k]); p[2 * (k - 1) + 1] = ZIM(pk[k]); }
    }
    free(cf); free(coef); free(pk);
    return rc;
}
