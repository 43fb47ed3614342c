// Double-double subset terms of the power-trace loop hafnian (the extended
// precision path).  Same mathematics as the FP64 per-subset kernels -- the
// bordered matrix C' = [[0, d_S^T], [X_S d_S, C]], its Householder Hessenberg
// form, La Budde over trailing blocks for det(xI - C) and det(xI - C'), then
// Newton's identities, the loop series and the exponential series -- but every
// operation in double-double (dd.h), with a simple layout: one workgroup of
// 256 threads per subset, the (m + 1) x (m + 1) matrix resident in LDS.
// The paper computes in x87 long double (64-bit significand); this path carries
// about 106 bits.
#include <hip/hip_runtime.h>

#include "dd.h"
#include "lhaf_kernels.h"

namespace gbs {

namespace {

constexpr int kDdThreads = 256;
constexpr int kDdSlices = kDdThreads / 64;  // row / term slices of the dot products
constexpr int kDdScratch = 448;             // cdd slots shared by the three phases

__device__ __forceinline__ cdd ld2(const double2 a) { return cdd_make(a.x, a.y); }

// Order LDS traffic between the lanes of one wavefront (no block barrier).
__device__ __forceinline__ void wave_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t unrank_colex_dd(uint64_t rank, int n, int s, const uint64_t* __restrict__ binom) {
    uint64_t mask = 0;
    int c = n - 1;
    for (int i = s; i >= 1; --i) {
        while (binom[c * kBinomStride + i] > rank) --c;
        mask |= 1ull << c;
        rank -= binom[c * kBinomStride + i];
        --c;
    }
    return mask;
}

__device__ __forceinline__ double shfl_xor_dbl(double x, int m) {
    const int lo = __shfl_xor(__double2loint(x), m);
    const int hi = __shfl_xor(__double2hiint(x), m);
    return __hiloint2double(hi, lo);
}

// Fixed-order butterfly sum over the 64 lanes of a wavefront; every lane ends
// with the same value (each pair is combined as lower lane + upper lane).
__device__ __forceinline__ cdd wave_sum_cdd(cdd x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        cdd y{dd{shfl_xor_dbl(x.re.hi, off), shfl_xor_dbl(x.re.lo, off)},
              dd{shfl_xor_dbl(x.im.hi, off), shfl_xor_dbl(x.im.lo, off)}};
        x = (lane & off) ? cdd_add(y, x) : cdd_add(x, y);
    }
    return x;
}

}  // namespace

int dd_lds_cdd_count(int m, int D) {
    const int K = m + 1, RS = D + 1;
    return K * K + RS * RS + kDdScratch;
}

size_t dd_lds_bytes(int m, int D) { return sizeof(cdd) * (size_t)dd_lds_cdd_count(m, D) + 64 * sizeof(int) + 64; }

namespace {

// One workgroup per subset of size s (m = 2s): writes its signed term t_S
// (double-double complex) to terms[g].
__global__ void __launch_bounds__(kDdThreads) charpoly_dd_kernel(const double2* __restrict__ A0,
                                                                 const double2* __restrict__ dvec, int Np, int s,
                                                                 uint64_t rank0, const uint64_t* __restrict__ masks,
                                                                 const uint64_t* __restrict__ binom, int D,
                                                                 double sign, cdd* __restrict__ terms) {
    extern __shared__ cdd lds_dd[];
    const int t = threadIdx.x;
    const int lane = t & 63, slice = t >> 6;
    const int n = Np >> 1, m = 2 * s, K = m + 1, RS = D + 1;
    cdd* H = lds_dd;            // K x K, row-major
    cdd* ring = H + K * K;      // RS x RS: coefficient d of P_q at ring[(q % RS) * RS + d]
    cdd* scr = ring + RS * RS;  // phase scratch
    int* idx = reinterpret_cast<int*>(scr + kDdScratch);
    dd* scal = reinterpret_cast<dd*>(idx + 64);  // tau of column c at [c & 1]

    const uint64_t g = blockIdx.x;
    const uint64_t mask = masks ? masks[g] : unrank_colex_dd(rank0 + g, n, s, binom);
    if (t < n && ((mask >> t) & 1ull)) {
        const int pos = __popcll(mask & ((1ull << t) - 1ull));
        idx[pos] = t;
        idx[pos + s] = t + n;
    }
    __syncthreads();
    // C' = [[0, d_S^T], [X_S d_S, X_S A0_S]]
    for (int e = t; e < K * K; e += kDdThreads) {
        const int r = e / K, c = e - r * K;
        cdd v = cdd_zero();
        if (r == 0 && c > 0) {
            v = ld2(dvec[idx[c - 1]]);
        } else if (r > 0) {
            const int rr = r - 1, xr = (rr < s) ? rr + s : rr - s;
            v = (c == 0) ? ld2(dvec[idx[xr]]) : ld2(A0[(int64_t)idx[xr] * Np + idx[c - 1]]);
        }
        H[e] = v;
    }
    __syncthreads();

    // ---- Householder Hessenberg reduction of C' ----
    cdd* v = scr;          // 64: reflector (scaled by tau in v2)
    cdd* v2 = scr + 64;    // 64: tau v
    cdd* part = scr + 128; // kDdSlices x 64
    for (int c = 0; c + 2 < K; ++c) {
        const int L = K - c - 1;  // rows / columns c+1..K-1
        // norm of x = H[c+1.., c]
        if (slice == 0) {
            const dd a2 = (lane < L) ? cdd_abs2(H[(c + 1 + lane) * K + c]) : dd{0.0, 0.0};
            const cdd tot = wave_sum_cdd(cdd{a2, dd{0.0, 0.0}});
            if (lane == 0) {
                const dd xn = dd_sqrt(tot.re);
                const cdd x0 = H[(c + 1) * K + c];
                const dd a0 = dd_sqrt(cdd_abs2(x0));
                if (xn.hi == 0.0) {
                    scal[c & 1] = dd{0.0, 0.0};
                    v[0] = cdd_zero();
                } else {
                    // phase of x0 (1 when x0 = 0); alpha = -phase |x|; v0 = x0 - alpha = phase (|x0| + |x|)
                    cdd ph = cdd_make(1.0, 0.0);
                    if (a0.hi != 0.0) {
                        const dd ia = dd_div(dd_make(1.0), a0);
                        ph = cdd_mul_dd(x0, ia);
                    }
                    const dd sum = dd_add(a0, xn);
                    v[0] = cdd_mul_dd(ph, sum);
                    scal[c & 1] = dd_div(dd_make(1.0), dd_mul(xn, sum));
                    const cdd alpha = cdd_mul_dd(ph, dd_neg(xn));
                    H[(c + 1) * K + c] = alpha;
                }
            }
            if (lane >= 1 && lane < L) v[lane] = H[(c + 1 + lane) * K + c];
        }
        __syncthreads();
        // tau is double-buffered: a wave that skips this column may still be
        // reading it while wave 0 already writes the next column's
        const dd tau = scal[c & 1];
        if (tau.hi == 0.0) continue;  // x = 0: already reduced (uniform across the block)
        if (t < L) v2[t] = cdd_mul_dd(v[t], tau);
        if (t >= 1 && t < L) H[(c + 1 + t) * K + c] = cdd_zero();
        // left: w_j = sum_i conj(v_i) H[c+1+i][c+1+j]
        if (lane < L) {
            cdd acc = cdd_zero();
            for (int i = slice; i < L; i += kDdSlices) acc = cdd_add(acc, cdd_cmul(v[i], H[(c + 1 + i) * K + c + 1 + lane]));
            part[slice * 64 + lane] = acc;
        }
        __syncthreads();
        cdd* w = scr + 128 + kDdSlices * 64;  // 64
        if (t < L) {
            cdd acc = part[t];
            for (int q = 1; q < kDdSlices; ++q) acc = cdd_add(acc, part[q * 64 + t]);
            w[t] = acc;
        }
        __syncthreads();
        for (int e = t; e < L * L; e += kDdThreads) {
            const int i = e / L, j = e - i * L;
            cdd& h = H[(c + 1 + i) * K + c + 1 + j];
            h = cdd_sub(h, cdd_mul(v2[i], w[j]));
        }
        __syncthreads();
        // right: u_i = sum_j H[i][c+1+j] v_j over all rows i
        if (lane < K) {
            cdd acc = cdd_zero();
            for (int j = slice; j < L; j += kDdSlices) acc = cdd_add(acc, cdd_mul(H[lane * K + c + 1 + j], v[j]));
            part[slice * 64 + lane] = acc;
        }
        __syncthreads();
        if (t < K) {
            cdd acc = part[t];
            for (int q = 1; q < kDdSlices; ++q) acc = cdd_add(acc, part[q * 64 + t]);
            w[t] = acc;
        }
        __syncthreads();
        for (int e = t; e < K * L; e += kDdThreads) {
            const int i = e / L, j = e - i * L;
            cdd& h = H[i * K + c + 1 + j];
            h = cdd_sub(h, cdd_mul(w[i], cdd_conj(v2[j])));
        }
        __syncthreads();
    }

    // ---- La Budde over trailing blocks: P_r(x) = det(xI - H[r:, r:]) ----
    // P_r = (x - h_rr) P_{r+1} - sum_{j>r} h_rj (prod_{i=r}^{j-1} h_{i+1,i}) P_{j+1};
    // coefficient d of P_q is that of x^{K - q - d}; only d <= D is kept.
    cdd* bp = scr;              // 2 x 64 ping-pong: prod_{i=r}^{r+o-1} beta_i at [o]
    cdd* gv = scr + 128;        // 64: h_{r, r+o} * bp[o]
    cdd* lp = scr + 192;        // kDdSlices x 64 partial sums (kDdScratch >= 192 + 4 * 64 - 64 checked below)
    for (int e = t; e < RS * RS; e += kDdThreads) ring[e] = cdd_zero();
    __syncthreads();
    if (t == 0) ring[(K % RS) * RS] = cdd_make(1.0, 0.0);
    __syncthreads();
    int cur = 0;
    for (int r = K - 1; r >= 0; --r) {
        const int omax = min(D - 1, K - 1 - r);  // offsets o = j - r with a possible term
        cdd* bo = bp + (cur ^ 1) * 64;        // previous step's products (offsets shifted by one)
        cdd* bn = bp + cur * 64;
        if (t >= 1 && t <= omax) {
            const cdd beta = H[(r + 1) * K + r];
            const cdd b = (t == 1) ? beta : cdd_mul(beta, bo[t - 1]);
            bn[t] = b;
            gv[t] = cdd_mul(H[r * K + r + t], b);
        }
        __syncthreads();
        const int deg = K - r;  // degree of P_r
        // partial sums of the terms of coefficient d = lane, offsets o = slice + 1 + 4k
        if (lane <= D && lane <= deg) {
            cdd acc = cdd_zero();
            for (int o = slice + 1; o <= min(lane - 1, omax); o += kDdSlices) {
                const int d2 = lane - o - 1;           // coefficient of P_{r+o+1}
                if (d2 <= K - 1 - (r + o))
                    acc = cdd_add(acc, cdd_mul(gv[o], ring[((r + o + 1) % RS) * RS + d2]));
            }
            lp[slice * 64 + lane] = acc;
        }
        __syncthreads();
        if (t <= D) {
            cdd val = cdd_zero();
            if (t <= deg) {
                const cdd* prev = ring + ((r + 1) % RS) * RS;
                if (t <= deg - 1) val = prev[t];
                if (t >= 1) val = cdd_sub(val, cdd_mul(H[r * K + r], prev[t - 1]));
                cdd acc = lp[t];
                for (int q = 1; q < kDdSlices; ++q) acc = cdd_add(acc, lp[q * 64 + t]);
                val = cdd_sub(val, acc);
            }
            ring[(r % RS) * RS + t] = val;
        }
        cur ^= 1;
        __syncthreads();
    }

    // ---- series (one wavefront): Newton, loop series, exp ----
    if (slice == 0) {
        const cdd* R = ring + (1 % RS) * RS;   // det(xI - C)
        const cdd* Rp = ring;                  // det(xI - C'), row 0
        cdd* Ls = scr;                         // 64
        cdd* ps = scr + 64;
        cdd* cs = scr + 128;
        cdd* es = scr + 192;
        if (lane == 0) es[0] = cdd_make(1.0, 0.0);
        const int nn = D - 1;  // = n
        for (int k = 1; k <= nn; ++k) {
            cdd a = cdd_zero(), b = cdd_zero();
            if (lane >= 1 && lane < k) {
                a = cdd_mul(R[lane], Ls[k - lane]);
                b = cdd_mul(R[lane], ps[k - lane]);
            }
            a = wave_sum_cdd(a);
            b = wave_sum_cdd(b);
            const cdd Lk = cdd_sub(cdd_sub(R[k + 1], Rp[k + 1]), a);
            const cdd pk = cdd_sub(cdd_mul_d(R[k], -(double)k), b);
            const cdd ck = cdd_add(cdd{dd_div(pk.re, dd_make(2.0 * k)), dd_div(pk.im, dd_make(2.0 * k))},
                                   cdd_mul_d(Lk, 0.5));
            if (lane == 0) {
                Ls[k] = Lk;
                ps[k] = pk;
                cs[k] = ck;
            }
            // e_k = (1/k) sum_{j=1..k} j c_j e_{k-j}
            cdd q = cdd_zero();
            if (lane >= 1 && lane <= k) {
                const cdd cj = (lane == k) ? ck : cs[lane];
                q = cdd_mul(cdd_mul_d(cj, (double)lane), es[k - lane]);
            }
            q = wave_sum_cdd(q);
            if (lane == 0) es[k] = cdd{dd_div(q.re, dd_make((double)k)), dd_div(q.im, dd_make((double)k))};
            wave_order();  // lane 0's writes are read by the other lanes at the next k
        }
        if (lane == 0) terms[g] = cdd_mul_d(es[nn], sign);
    }
}

// Block b sums terms [b * 64 * per, (b + 1) * 64 * per) in a fixed order:
// lane l takes terms b * 64 * per + q * 64 + l, then a fixed butterfly.
__global__ void __launch_bounds__(64) dd_block_reduce_kernel(const cdd* __restrict__ terms, uint64_t count, int per,
                                                             double* __restrict__ partials,
                                                             double2* __restrict__ terms_out) {
    const int lane = threadIdx.x;
    cdd acc = cdd_zero();
    double ab = 0.0;
    const uint64_t base = (uint64_t)blockIdx.x * 64 * per;
    for (int q = 0; q < per; ++q) {
        const uint64_t g = base + (uint64_t)q * 64 + lane;
        if (g < count) {
            const cdd x = terms[g];
            if (terms_out) terms_out[g] = make_double2(x.re.hi + x.re.lo, x.im.hi + x.im.lo);
            acc = cdd_add(acc, x);
            ab += sqrt(x.re.hi * x.re.hi + x.im.hi * x.im.hi);
        }
    }
    acc = wave_sum_cdd(acc);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double y = shfl_xor_dbl(ab, off);
        ab = (lane & off) ? y + ab : ab + y;
    }
    if (lane == 0) {
        double* o = partials + 5 * (uint64_t)blockIdx.x;
        o[0] = acc.re.hi;
        o[1] = acc.re.lo;
        o[2] = acc.im.hi;
        o[3] = acc.im.lo;
        o[4] = ab;
    }
}

// Fixed-order dd sum of np partial records (re.hi, re.lo, im.hi, im.lo, |t|).
__global__ void __launch_bounds__(64) dd_final_reduce_kernel(const double* __restrict__ partials, int64_t np,
                                                             double2* __restrict__ out_hi,
                                                             double2* __restrict__ out_lo, double* __restrict__ abs_out) {
    const int lane = threadIdx.x;
    cdd acc = cdd_zero();
    double ab = 0.0;
    for (int64_t i = lane; i < np; i += 64) {
        const double* p = partials + 5 * i;
        acc = cdd_add(acc, cdd{dd{p[0], p[1]}, dd{p[2], p[3]}});
        ab += p[4];
    }
    acc = wave_sum_cdd(acc);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double y = shfl_xor_dbl(ab, off);
        ab = (lane & off) ? y + ab : ab + y;
    }
    if (lane == 0) {
        out_hi[0] = make_double2(acc.re.hi, acc.im.hi);
        if (out_lo) out_lo[0] = make_double2(acc.re.lo, acc.im.lo);
        if (abs_out) abs_out[0] = ab;
    }
}

}  // namespace

hipError_t launch_charpoly_dd(const double2* A0, const double2* dvec, int Np, int s, uint64_t rank0, uint64_t count,
                              const uint64_t* masks, const uint64_t* binom, int D, double sign, void* terms,
                              hipStream_t st) {
    if (count == 0) return hipSuccess;
    const int m = 2 * s;
    if (s < 1 || m > 2 * kMaxDdPairs || D < 2 || D > kMaxDdPairs + 1 || count > (uint64_t)INT32_MAX)
        return hipErrorInvalidValue;
    static_assert(kDdScratch >= 192 + kDdSlices * 64, "La Budde scratch");
    static_assert(kDdScratch >= 128 + kDdSlices * 64 + 64, "Householder scratch");
    const size_t lds = dd_lds_bytes(m, D);
    static bool attr = false;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&charpoly_dd_kernel),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)dd_lds_bytes(2 * kMaxDdPairs, kMaxDdPairs + 1));
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(charpoly_dd_kernel, dim3((unsigned)count), dim3(kDdThreads), lds, st, A0, dvec, Np, s, rank0,
                       masks, binom, D, sign, static_cast<cdd*>(terms));
    return hipGetLastError();
}

hipError_t launch_dd_block_reduce(const void* terms, uint64_t count, int per, double* partials, double2* terms_out,
                                  hipStream_t st) {
    if (count == 0) return hipSuccess;
    const uint64_t nb = (count + 64ull * per - 1) / (64ull * per);
    hipLaunchKernelGGL(dd_block_reduce_kernel, dim3((unsigned)nb), dim3(64), 0, st, static_cast<const cdd*>(terms),
                       count, per, partials, terms_out);
    return hipGetLastError();
}

hipError_t launch_dd_final_reduce(const double* partials, int64_t np, double2* out_hi, double2* out_lo, double* abs_out,
                                  hipStream_t st) {
    hipLaunchKernelGGL(dd_final_reduce_kernel, dim3(1), dim3(64), 0, st, partials, np, out_hi, out_lo, abs_out);
    return hipGetLastError();
}

}  // namespace gbs
