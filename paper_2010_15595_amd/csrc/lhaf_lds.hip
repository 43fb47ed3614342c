// Subset terms of the power-trace loop hafnian with the subset's matrix
// resident in LDS: one workgroup of 256 threads per subset.  The mathematics is
// that of the register-tiled FP64 kernels -- the bordered matrix
// C' = [[0, d_S^T], [X_S d_S, C]], its Householder Hessenberg form H', the
// characteristic polynomials det(xI - C) and det(xI - C'), then Newton's
// identities, the loop series and the exponential series -- in one of two
// arithmetics and with one of two ways to get the characteristic polynomials:
//   * double-double (dd.h, ~106-bit significand): the extended precision path
//     (the paper's CPU code uses x87 long double, Sec. IV);
//   * FP64: a plain reference layout for comparing methods;
//   * La Budde over trailing blocks of H' (the method the paper uses), or
//   * eigenvalues of H'[1:, 1:] and H' by the shifted QR algorithm, multiplied
//     out into the polynomials: the diagonalisation the paper compares La
//     Budde against (Sec. IV).
#include <hip/hip_runtime.h>

#include "dd.h"
#include "lhaf_kernels.h"

namespace gbs {

namespace {

constexpr int kLdsThreads = 256;
constexpr int kSlices = kLdsThreads / 64;  // row / term slices of the dot products
constexpr int kScratch = 456;              // complex slots shared by the phases
constexpr int kMaxQrSweeps = 30;           // per eigenvalue, before the subset is marked failed

__device__ __forceinline__ double shfl_xor_dbl(double x, int m) {
    const int lo = __shfl_xor(__double2loint(x), m);
    const int hi = __shfl_xor(__double2hiint(x), m);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double shfl_up_dbl(double x, int d) {
    const int lo = __shfl_up(__double2loint(x), d);
    const int hi = __shfl_up(__double2hiint(x), d);
    return __hiloint2double(hi, lo);
}

// Arithmetic policies: complex type C over real type R.
struct ArDD {
    using R = dd;
    using C = cdd;
    static constexpr double eps = 1e-31;
    __device__ static C zero() { return cdd_zero(); }
    __device__ static C make(double re, double im) { return cdd_make(re, im); }
    __device__ static C ld(double2 a) { return cdd_make(a.x, a.y); }
    __device__ static C add(C a, C b) { return cdd_add(a, b); }
    __device__ static C sub(C a, C b) { return cdd_sub(a, b); }
    __device__ static C mul(C a, C b) { return cdd_mul(a, b); }
    __device__ static C cmul(C a, C b) { return cdd_cmul(a, b); }
    __device__ static C conj(C a) { return cdd_conj(a); }
    __device__ static C mul_r(C a, R b) { return cdd_mul_dd(a, b); }
    __device__ static C mul_d(C a, double b) { return cdd_mul_d(a, b); }
    __device__ static C div_d(C a, double b) { return C{dd_div(a.re, dd_make(b)), dd_div(a.im, dd_make(b))}; }
    __device__ static R abs2(C a) { return cdd_abs2(a); }
    __device__ static R r_zero() { return dd{0.0, 0.0}; }
    __device__ static R r_one() { return dd{1.0, 0.0}; }
    __device__ static R r_add(R a, R b) { return dd_add(a, b); }
    __device__ static R r_mul(R a, R b) { return dd_mul(a, b); }
    __device__ static R r_div(R a, R b) { return dd_div(a, b); }
    __device__ static R r_sqrt(R a) { return dd_sqrt(a); }
    __device__ static R r_neg(R a) { return dd_neg(a); }
    __device__ static double hi(R a) { return a.hi; }
    __device__ static C shfl_xor(C x, int off) {
        return C{dd{shfl_xor_dbl(x.re.hi, off), shfl_xor_dbl(x.re.lo, off)},
                 dd{shfl_xor_dbl(x.im.hi, off), shfl_xor_dbl(x.im.lo, off)}};
    }
    __device__ static C shfl_up(C x, int d) {
        return C{dd{shfl_up_dbl(x.re.hi, d), shfl_up_dbl(x.re.lo, d)},
                 dd{shfl_up_dbl(x.im.hi, d), shfl_up_dbl(x.im.lo, d)}};
    }
    __device__ static cdd to_dd(C a) { return a; }
};

struct cf64 {
    double re, im;
};

struct ArF64 {
    using R = double;
    using C = cf64;
    static constexpr double eps = 2.3e-16;
    __device__ static C zero() { return C{0.0, 0.0}; }
    __device__ static C make(double re, double im) { return C{re, im}; }
    __device__ static C ld(double2 a) { return C{a.x, a.y}; }
    __device__ static C add(C a, C b) { return C{a.re + b.re, a.im + b.im}; }
    __device__ static C sub(C a, C b) { return C{a.re - b.re, a.im - b.im}; }
    __device__ static C mul(C a, C b) { return C{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
    __device__ static C cmul(C a, C b) { return C{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }
    __device__ static C conj(C a) { return C{a.re, -a.im}; }
    __device__ static C mul_r(C a, R b) { return C{a.re * b, a.im * b}; }
    __device__ static C mul_d(C a, double b) { return C{a.re * b, a.im * b}; }
    __device__ static C div_d(C a, double b) { return C{a.re / b, a.im / b}; }
    __device__ static R abs2(C a) { return a.re * a.re + a.im * a.im; }
    __device__ static R r_zero() { return 0.0; }
    __device__ static R r_one() { return 1.0; }
    __device__ static R r_add(R a, R b) { return a + b; }
    __device__ static R r_mul(R a, R b) { return a * b; }
    __device__ static R r_div(R a, R b) { return a / b; }
    __device__ static R r_sqrt(R a) { return sqrt(a); }
    __device__ static R r_neg(R a) { return -a; }
    __device__ static double hi(R a) { return a; }
    __device__ static C shfl_xor(C x, int off) { return C{shfl_xor_dbl(x.re, off), shfl_xor_dbl(x.im, off)}; }
    __device__ static C shfl_up(C x, int d) { return C{shfl_up_dbl(x.re, d), shfl_up_dbl(x.im, d)}; }
    __device__ static cdd to_dd(C a) { return cdd_make(a.re, a.im); }
};

// Order LDS traffic between the lanes of one wavefront (no block barrier).
__device__ __forceinline__ void wave_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t unrank_colex_lds(uint64_t rank, int n, int s, const uint64_t* __restrict__ binom) {
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

// Fixed-order butterfly sum over the 64 lanes of a wavefront; every lane ends
// with the same value (each pair is combined as lower lane + upper lane).
template <class Ar>
__device__ __forceinline__ typename Ar::C wave_sum(typename Ar::C x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const typename Ar::C y = Ar::shfl_xor(x, off);
        x = (lane & off) ? Ar::add(y, x) : Ar::add(x, y);
    }
    return x;
}

// Eigenvalues of the upper Hessenberg q x q matrix W (row stride q, destroyed)
// by the single-shift complex QR algorithm with Wilkinson shifts and
// deflation on negligible subdiagonal entries (Golub and Van Loan, ch. 7),
// run by one wavefront.  Eigenvalues go to ev[0..q).  Returns false when an
// eigenvalue needs more than kMaxQrSweeps sweeps.
template <class Ar>
__device__ bool qr_eigenvalues(typename Ar::C* W, int q, typename Ar::C* ev, typename Ar::C* rot, int* flag) {
    using C = typename Ar::C;
    const int lane = threadIdx.x & 63;
    int hi = q - 1, sweeps = 0;
    while (hi >= 0) {
        if (hi == 0) {
            if (lane == 0) ev[0] = W[0];
            break;
        }
        // lowest l such that W[l..hi] has no negligible subdiagonal entry
        if (lane == 0) {
            int l = hi;
            while (l > 0) {
                const double sub = Ar::hi(Ar::abs2(W[l * q + l - 1]));
                const double dg = sqrt(Ar::hi(Ar::abs2(W[l * q + l]))) + sqrt(Ar::hi(Ar::abs2(W[(l - 1) * q + l - 1])));
                if (sqrt(sub) <= Ar::eps * dg) {
                    W[l * q + l - 1] = Ar::zero();
                    break;
                }
                --l;
            }
            flag[0] = l;
        }
        wave_order();
        const int l = __builtin_amdgcn_readfirstlane(flag[0]);
        if (l == hi) {
            if (lane == 0) ev[hi] = W[hi * q + hi];
            --hi;
            sweeps = 0;
            wave_order();
            continue;
        }
        if (++sweeps > kMaxQrSweeps) return false;
        // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block closest to its last entry;
        // an exceptional shift every tenth sweep breaks cycles
        if (lane == 0) {
            const C a = W[(hi - 1) * q + hi - 1], b = W[(hi - 1) * q + hi], c = W[hi * q + hi - 1], d = W[hi * q + hi];
            C mu = d;
            if (sweeps % 10 == 0) {
                mu = Ar::add(d, Ar::mul_d(Ar::make(sqrt(Ar::hi(Ar::abs2(c))), 0.0), 0.75));
            } else {
                // roots of x^2 - (a + d) x + (ad - bc): mu = d - bc / (h + sign(h) sqrt(h^2 + bc)), h = (a - d)/2
                const C h = Ar::mul_d(Ar::sub(a, d), 0.5);
                const C bc = Ar::mul(b, c);
                const C disc = Ar::add(Ar::mul(h, h), bc);
                // principal square root of disc in the working precision of its high parts
                const double dr = Ar::hi(disc.re), di = Ar::hi(disc.im);
                const double r = sqrt(dr * dr + di * di);
                double sr = sqrt(0.5 * (r + dr)), si = sqrt(0.5 * (r - dr));
                if (di < 0) si = -si;
                C sq = Ar::make(sr, si);
                C den = Ar::add(h, sq);
                if (Ar::hi(h.re) * sr + Ar::hi(h.im) * si < 0) den = Ar::sub(h, sq);
                const double dn = Ar::hi(Ar::abs2(den));
                if (dn > 0.0) {
                    // bc / den = bc conj(den) / |den|^2
                    const C f = Ar::mul_r(Ar::cmul(den, bc), Ar::r_div(Ar::r_one(), Ar::abs2(den)));
                    mu = Ar::sub(d, f);
                }
            }
            rot[2 * 64] = mu;
        }
        wave_order();
        const C mu = rot[2 * 64];
        for (int i = l + lane; i <= hi; i += 64) W[i * q + i] = Ar::sub(W[i * q + i], mu);
        wave_order();
        // left: Givens rotations G_j zero W[j+1][j], j = l..hi-1
        for (int j = l; j < hi; ++j) {
            if (lane == 0) {
                const C a = W[j * q + j], b = W[(j + 1) * q + j];
                const typename Ar::R na2 = Ar::abs2(a);
                const typename Ar::R n = Ar::r_sqrt(Ar::r_add(na2, Ar::abs2(b)));
                C cs = Ar::make(1.0, 0.0), sn = Ar::zero();
                if (Ar::hi(n) != 0.0) {
                    const typename Ar::R in = Ar::r_div(Ar::r_one(), n);
                    if (Ar::hi(na2) == 0.0) {
                        cs = Ar::zero();
                        sn = Ar::mul_r(Ar::conj(b), in);
                    } else {
                        const typename Ar::R na = Ar::r_sqrt(na2);
                        cs = C{Ar::r_mul(na, in), Ar::r_zero()};
                        // s = (a / |a|) conj(b) / n
                        sn = Ar::mul_r(Ar::mul(a, Ar::conj(b)), Ar::r_div(in, na));
                    }
                }
                rot[j - l] = cs;
                rot[64 + j - l] = sn;
            }
            wave_order();
            const C cs = rot[j - l], sn = rot[64 + j - l];
            for (int k = j + lane; k <= hi; k += 64) {
                const C x = W[j * q + k], y = W[(j + 1) * q + k];
                W[j * q + k] = Ar::add(Ar::mul(cs, x), Ar::mul(sn, y));
                W[(j + 1) * q + k] = Ar::sub(Ar::mul(cs, y), Ar::cmul(sn, x));
            }
            wave_order();
        }
        // right: W <- W G_j^H, j = l..hi-1 (rows l..j+1)
        for (int j = l; j < hi; ++j) {
            const C cs = rot[j - l], sn = rot[64 + j - l];
            for (int k = l + lane; k <= j + 1; k += 64) {
                const C x = W[k * q + j], y = W[k * q + j + 1];
                W[k * q + j] = Ar::add(Ar::mul(cs, x), Ar::cmul(sn, y));
                W[k * q + j + 1] = Ar::sub(Ar::mul(cs, y), Ar::mul(sn, x));
            }
            wave_order();
        }
        for (int i = l + lane; i <= hi; i += 64) W[i * q + i] = Ar::add(W[i * q + i], mu);
        wave_order();
    }
    return true;
}

// det(xI - M) leading coefficients 0..D from the eigenvalues ev[0..q) of M:
// prod_i (1 - ev_i eta) multiplied out, lane d holding coefficient d.
template <class Ar>
__device__ void poly_from_eigenvalues(const typename Ar::C* ev, int q, int D, typename Ar::C* out) {
    using C = typename Ar::C;
    const int lane = threadIdx.x & 63;
    C coef = (lane == 0) ? Ar::make(1.0, 0.0) : Ar::zero();
    for (int i = 0; i < q; ++i) {
        const C prev = Ar::shfl_up(coef, 1);
        if (lane >= 1) coef = Ar::sub(coef, Ar::mul(ev[i], prev));
    }
    if (lane <= D) out[lane] = coef;
}

}  // namespace

int lds_cx_count(int m, int D, int method) {
    const int K = m + 1, RS = D + 1;
    return K * K * (method == kCharpolyEigen ? 2 : 1) + RS * RS + kScratch;
}

size_t lds_bytes(int m, int D, int prec_dd, int method) {
    return (prec_dd ? sizeof(cdd) : sizeof(cf64)) * (size_t)lds_cx_count(m, D, method) + 64 * sizeof(int) + 64;
}

size_t dd_lds_bytes(int m, int D) { return lds_bytes(m, D, 1, kCharpolyLaBudde); }

namespace {

// One workgroup per subset of size s (m = 2s): writes its signed term t_S to
// terms[g] (type Ar::C); a subset whose QR iteration fails gets NaN.
template <class Ar, int METHOD>
__global__ void __launch_bounds__(kLdsThreads) charpoly_lds_kernel(const double2* __restrict__ A0,
                                                                   const double2* __restrict__ dvec, int Np, int s,
                                                                   uint64_t rank0, const uint64_t* __restrict__ masks,
                                                                   const uint64_t* __restrict__ binom, int D,
                                                                   double sign, typename Ar::C* __restrict__ terms) {
    using C = typename Ar::C;
    using R = typename Ar::R;
    extern __shared__ double4 lds_raw[];
    C* lds = reinterpret_cast<C*>(lds_raw);
    const int t = threadIdx.x;
    const int lane = t & 63, slice = t >> 6;
    const int n = Np >> 1, m = 2 * s, K = m + 1, RS = D + 1;
    C* H = lds;                                                  // K x K, row-major
    C* Wq = H + K * K;                                           // K x K work copy (eigenvalue method)
    C* ring = Wq + (METHOD == kCharpolyEigen ? K * K : 0);       // RS x RS
    C* scr = ring + RS * RS;                                     // phase scratch
    int* idx = reinterpret_cast<int*>(scr + kScratch);
    R* scal = reinterpret_cast<R*>(idx + 64);                    // tau of column c at [c & 1]

    const uint64_t g = blockIdx.x;
    const uint64_t mask = masks ? masks[g] : unrank_colex_lds(rank0 + g, n, s, binom);
    if (t < n && ((mask >> t) & 1ull)) {
        const int pos = __popcll(mask & ((1ull << t) - 1ull));
        idx[pos] = t;
        idx[pos + s] = t + n;
    }
    __syncthreads();
    // C' = [[0, d_S^T], [X_S d_S, X_S A0_S]]
    for (int e = t; e < K * K; e += kLdsThreads) {
        const int r = e / K, c = e - r * K;
        C v = Ar::zero();
        if (r == 0 && c > 0) {
            v = Ar::ld(dvec[idx[c - 1]]);
        } else if (r > 0) {
            const int rr = r - 1, xr = (rr < s) ? rr + s : rr - s;
            v = (c == 0) ? Ar::ld(dvec[idx[xr]]) : Ar::ld(A0[(int64_t)idx[xr] * Np + idx[c - 1]]);
        }
        H[e] = v;
    }
    __syncthreads();

    // ---- Householder Hessenberg reduction of C' ----
    C* v = scr;          // 64: reflector
    C* v2 = scr + 64;    // 64: tau v
    C* part = scr + 128; // kSlices x 65 (row partials; K <= 65 rows)
    C* w = scr + 128 + kSlices * 65;  // 65
    for (int c = 0; c + 2 < K; ++c) {
        const int L = K - c - 1;  // rows / columns c+1..K-1
        if (slice == 0) {
            const R a2 = (lane < L) ? Ar::abs2(H[(c + 1 + lane) * K + c]) : Ar::r_zero();
            const C tot = wave_sum<Ar>(C{a2, Ar::r_zero()});
            if (lane == 0) {
                const R xn = Ar::r_sqrt(tot.re);
                const C x0 = H[(c + 1) * K + c];
                const R a0 = Ar::r_sqrt(Ar::abs2(x0));
                if (Ar::hi(xn) == 0.0) {
                    scal[c & 1] = Ar::r_zero();
                    v[0] = Ar::zero();
                } else {
                    // phase of x0 (1 when x0 = 0); alpha = -phase |x|; v0 = x0 - alpha = phase (|x0| + |x|)
                    C ph = Ar::make(1.0, 0.0);
                    if (Ar::hi(a0) != 0.0) ph = Ar::mul_r(x0, Ar::r_div(Ar::r_one(), a0));
                    const R sum = Ar::r_add(a0, xn);
                    v[0] = Ar::mul_r(ph, sum);
                    scal[c & 1] = Ar::r_div(Ar::r_one(), Ar::r_mul(xn, sum));
                    H[(c + 1) * K + c] = Ar::mul_r(ph, Ar::r_neg(xn));
                }
            }
            if (lane >= 1 && lane < L) v[lane] = H[(c + 1 + lane) * K + c];
        }
        __syncthreads();
        // tau is double-buffered: a wave that skips this column may still be
        // reading it while wave 0 already writes the next column's
        const R tau = scal[c & 1];
        if (Ar::hi(tau) == 0.0) continue;  // x = 0: already reduced (uniform across the block)
        if (t < L) v2[t] = Ar::mul_r(v[t], tau);
        if (t >= 1 && t < L) H[(c + 1 + t) * K + c] = Ar::zero();
        // left: w_j = sum_i conj(v_i) H[c+1+i][c+1+j]
        if (lane < L) {
            C acc = Ar::zero();
            for (int i = slice; i < L; i += kSlices) acc = Ar::add(acc, Ar::cmul(v[i], H[(c + 1 + i) * K + c + 1 + lane]));
            part[slice * 64 + lane] = acc;
        }
        __syncthreads();
        if (t < L) {
            C acc = part[t];
            for (int q = 1; q < kSlices; ++q) acc = Ar::add(acc, part[q * 64 + t]);
            w[t] = acc;
        }
        __syncthreads();
        for (int e = t; e < L * L; e += kLdsThreads) {
            const int i = e / L, j = e - i * L;
            C& h = H[(c + 1 + i) * K + c + 1 + j];
            h = Ar::sub(h, Ar::mul(v2[i], w[j]));
        }
        __syncthreads();
        // right: u_i = sum_j H[i][c+1+j] v_j over all rows i (K <= 65: lane l takes rows l and l + 64)
        for (int i = lane; i < K; i += 64) {
            C acc = Ar::zero();
            for (int j = slice; j < L; j += kSlices) acc = Ar::add(acc, Ar::mul(H[i * K + c + 1 + j], v[j]));
            part[slice * 65 + i] = acc;
        }
        __syncthreads();
        for (int i = t; i < K; i += kLdsThreads) {
            C acc = part[i];
            for (int q = 1; q < kSlices; ++q) acc = Ar::add(acc, part[q * 65 + i]);
            w[i] = acc;
        }
        __syncthreads();
        for (int e = t; e < K * L; e += kLdsThreads) {
            const int i = e / L, j = e - i * L;
            C& h = H[i * K + c + 1 + j];
            h = Ar::sub(h, Ar::mul(w[i], Ar::conj(v2[j])));
        }
        __syncthreads();
    }

    if constexpr (METHOD == kCharpolyLaBudde) {
        // ---- La Budde over trailing blocks: P_r(x) = det(xI - H[r:, r:]) ----
        // P_r = (x - h_rr) P_{r+1} - sum_{j>r} h_rj (prod_{i=r}^{j-1} h_{i+1,i}) P_{j+1};
        // coefficient d of P_q is that of x^{K - q - d}; only d <= D is kept.
        C* bp = scr;         // 2 x 64 ping-pong: prod_{i=r}^{r+o-1} beta_i at [o]
        C* gv = scr + 128;   // 64: h_{r, r+o} * bp[o]
        C* lp = scr + 192;   // kSlices x 64 partial sums
        for (int e = t; e < RS * RS; e += kLdsThreads) ring[e] = Ar::zero();
        __syncthreads();
        if (t == 0) ring[(K % RS) * RS] = Ar::make(1.0, 0.0);
        __syncthreads();
        int cur = 0;
        for (int r = K - 1; r >= 0; --r) {
            const int omax = min(D - 1, K - 1 - r);  // offsets o = j - r with a possible term
            C* bo = bp + (cur ^ 1) * 64;             // previous step's products (offsets shifted by one)
            C* bn = bp + cur * 64;
            if (t >= 1 && t <= omax) {
                const C beta = H[(r + 1) * K + r];
                const C b = (t == 1) ? beta : Ar::mul(beta, bo[t - 1]);
                bn[t] = b;
                gv[t] = Ar::mul(H[r * K + r + t], b);
            }
            __syncthreads();
            const int deg = K - r;  // degree of P_r
            // partial sums of the terms of coefficient d = lane, offsets o = slice + 1 + 4k
            if (lane <= D && lane <= deg) {
                C acc = Ar::zero();
                for (int o = slice + 1; o <= min(lane - 1, omax); o += kSlices) {
                    const int d2 = lane - o - 1;  // coefficient of P_{r+o+1}
                    if (d2 <= K - 1 - (r + o)) acc = Ar::add(acc, Ar::mul(gv[o], ring[((r + o + 1) % RS) * RS + d2]));
                }
                lp[slice * 64 + lane] = acc;
            }
            __syncthreads();
            if (t <= D) {
                C val = Ar::zero();
                if (t <= deg) {
                    const C* prev = ring + ((r + 1) % RS) * RS;
                    if (t <= deg - 1) val = prev[t];
                    if (t >= 1) val = Ar::sub(val, Ar::mul(H[r * K + r], prev[t - 1]));
                    C acc = lp[t];
                    for (int q = 1; q < kSlices; ++q) acc = Ar::add(acc, lp[q * 64 + t]);
                    val = Ar::sub(val, acc);
                }
                ring[(r % RS) * RS + t] = val;
            }
            cur ^= 1;
            __syncthreads();
        }
    } else {
        // ---- eigenvalues of H'[1:, 1:] (similar to C) and of H' (similar to C') ----
        if (slice != 0) return;  // one wavefront from here on; no block barrier follows
        C* ev = scr;             // 64 eigenvalues (K <= 64 + 1 handled by the lane loops)
        C* rot = scr + 128;      // Givens cosines [0, 64), sines [64, 128), shift [128]
        int* flag = idx;         // idx is no longer needed
        bool ok = true;
        // H'[1:, 1:] -> Wq (row stride m)
        for (int e = lane; e < m * m; e += 64) {
            const int r = e / m, c = e - r * m;
            Wq[e] = H[(r + 1) * K + c + 1];
        }
        wave_order();
        ok = qr_eigenvalues<Ar>(Wq, m, ev, rot, flag);
        wave_order();
        poly_from_eigenvalues<Ar>(ev, m, D, ring + (1 % RS) * RS);
        wave_order();
        if (ok) {
            for (int e = lane; e < K * K; e += 64) Wq[e] = H[e];
            wave_order();
            ok = qr_eigenvalues<Ar>(Wq, K, ev, rot, flag);
            wave_order();
            poly_from_eigenvalues<Ar>(ev, K, D, ring);
            wave_order();
        }
        if (!ok) {
            if (lane == 0) terms[g] = Ar::make(__builtin_nan(""), __builtin_nan(""));
            return;
        }
    }

    // ---- series (one wavefront): Newton, loop series, exp ----
    if (slice == 0) {
        const C* Rc = ring + (1 % RS) * RS;  // det(xI - C)
        const C* Rp = ring;                  // det(xI - C'), row 0
        C* Ls = scr + 192;                   // the eigenvalue method keeps ev and rot below 192
        C* ps = scr + 256;
        C* cs = scr + 320;
        C* es = scr + 384;
        if (lane == 0) es[0] = Ar::make(1.0, 0.0);
        wave_order();
        const int nn = D - 1;  // = n
        for (int k = 1; k <= nn; ++k) {
            C a = Ar::zero(), b = Ar::zero();
            if (lane >= 1 && lane < k) {
                a = Ar::mul(Rc[lane], Ls[k - lane]);
                b = Ar::mul(Rc[lane], ps[k - lane]);
            }
            a = wave_sum<Ar>(a);
            b = wave_sum<Ar>(b);
            const C Lk = Ar::sub(Ar::sub(Rc[k + 1], Rp[k + 1]), a);
            const C pk = Ar::sub(Ar::mul_d(Rc[k], -(double)k), b);
            const C ck = Ar::add(Ar::div_d(pk, 2.0 * k), Ar::mul_d(Lk, 0.5));
            if (lane == 0) {
                Ls[k] = Lk;
                ps[k] = pk;
                cs[k] = ck;
            }
            // e_k = (1/k) sum_{j=1..k} j c_j e_{k-j}
            C q = Ar::zero();
            if (lane >= 1 && lane <= k) {
                const C cj = (lane == k) ? ck : cs[lane];
                q = Ar::mul(Ar::mul_d(cj, (double)lane), es[k - lane]);
            }
            q = wave_sum<Ar>(q);
            if (lane == 0) es[k] = Ar::div_d(q, (double)k);
            wave_order();  // lane 0's writes are read by the other lanes at the next k
        }
        if (lane == 0) terms[g] = Ar::mul_d(es[nn], sign);
    }
}

// Block b sums terms [b * 64 * per, (b + 1) * 64 * per) in double-double in a
// fixed order: lane l takes terms b * 64 * per + q * 64 + l, then a fixed butterfly.
template <class Ar>
__global__ void __launch_bounds__(64) lds_block_reduce_kernel(const typename Ar::C* __restrict__ terms,
                                                              uint64_t count, int per, double* __restrict__ partials,
                                                              double2* __restrict__ terms_out) {
    const int lane = threadIdx.x;
    cdd acc = cdd_zero();
    double ab = 0.0;
    const uint64_t base = (uint64_t)blockIdx.x * 64 * per;
    for (int q = 0; q < per; ++q) {
        const uint64_t g = base + (uint64_t)q * 64 + lane;
        if (g < count) {
            const cdd x = Ar::to_dd(terms[g]);
            if (terms_out) terms_out[g] = make_double2(x.re.hi + x.re.lo, x.im.hi + x.im.lo);
            acc = cdd_add(acc, x);
            ab += sqrt(x.re.hi * x.re.hi + x.im.hi * x.im.hi);
        }
    }
    acc = wave_sum<ArDD>(acc);
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
    acc = wave_sum<ArDD>(acc);
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

template <class Ar, int METHOD>
hipError_t launch_lds_t(const double2* A0, const double2* dvec, int Np, int s, uint64_t rank0, uint64_t count,
                        const uint64_t* masks, const uint64_t* binom, int D, double sign, void* terms, size_t lds,
                        size_t lds_max, hipStream_t st) {
    // the dynamic-LDS limit is a per-device attribute of the kernel (callers hold the library lock)
    static bool attr[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (!attr[dev]) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&charpoly_lds_kernel<Ar, METHOD>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
        if (e != hipSuccess) return e;
        attr[dev] = true;
    }
    hipLaunchKernelGGL((charpoly_lds_kernel<Ar, METHOD>), dim3((unsigned)count), dim3(kLdsThreads), lds, st, A0, dvec,
                       Np, s, rank0, masks, binom, D, sign, static_cast<typename Ar::C*>(terms));
    return hipGetLastError();
}

}  // namespace

int lds_max_pairs(int prec_dd, int method) {
    if (method == kCharpolyEigen) return prec_dd ? 0 : 32;
    return prec_dd ? kMaxDdPairs : 32;
}

size_t lds_term_bytes(int prec_dd) { return prec_dd ? sizeof(cdd) : sizeof(cf64); }

hipError_t launch_charpoly_lds(int prec_dd, int method, const double2* A0, const double2* dvec, int Np, int s,
                               uint64_t rank0, uint64_t count, const uint64_t* masks, const uint64_t* binom, int D,
                               double sign, void* terms, hipStream_t st) {
    if (count == 0) return hipSuccess;
    const int m = 2 * s, maxp = lds_max_pairs(prec_dd, method);
    if (s < 1 || maxp == 0 || m > 2 * maxp || D < 2 || D > maxp + 1 || count > (uint64_t)INT32_MAX)
        return hipErrorInvalidValue;
    static_assert(kScratch >= 384 + 64, "series scratch");
    static_assert(kScratch >= 128 + kSlices * 65 + 65, "Householder scratch");
    const size_t lds = lds_bytes(m, D, prec_dd, method), lds_max = lds_bytes(2 * maxp, maxp + 1, prec_dd, method);
    if (lds_max > 160 * 1024) return hipErrorInvalidValue;
    if (prec_dd)
        return launch_lds_t<ArDD, kCharpolyLaBudde>(A0, dvec, Np, s, rank0, count, masks, binom, D, sign, terms, lds,
                                                    lds_max, st);
    if (method == kCharpolyEigen)
        return launch_lds_t<ArF64, kCharpolyEigen>(A0, dvec, Np, s, rank0, count, masks, binom, D, sign, terms, lds,
                                                   lds_max, st);
    return launch_lds_t<ArF64, kCharpolyLaBudde>(A0, dvec, Np, s, rank0, count, masks, binom, D, sign, terms, lds,
                                                 lds_max, st);
}

hipError_t launch_charpoly_dd(const double2* A0, const double2* dvec, int Np, int s, uint64_t rank0, uint64_t count,
                              const uint64_t* masks, const uint64_t* binom, int D, double sign, void* terms,
                              hipStream_t st) {
    return launch_charpoly_lds(1, kCharpolyLaBudde, A0, dvec, Np, s, rank0, count, masks, binom, D, sign, terms, st);
}

hipError_t launch_lds_block_reduce(int prec_dd, const void* terms, uint64_t count, int per, double* partials,
                                   double2* terms_out, hipStream_t st) {
    if (count == 0) return hipSuccess;
    const uint64_t nb = (count + 64ull * per - 1) / (64ull * per);
    if (prec_dd)
        hipLaunchKernelGGL(lds_block_reduce_kernel<ArDD>, dim3((unsigned)nb), dim3(64), 0, st,
                           static_cast<const cdd*>(terms), count, per, partials, terms_out);
    else
        hipLaunchKernelGGL(lds_block_reduce_kernel<ArF64>, dim3((unsigned)nb), dim3(64), 0, st,
                           static_cast<const cf64*>(terms), count, per, partials, terms_out);
    return hipGetLastError();
}

hipError_t launch_dd_block_reduce(const void* terms, uint64_t count, int per, double* partials, double2* terms_out,
                                  hipStream_t st) {
    return launch_lds_block_reduce(1, terms, count, per, partials, terms_out, st);
}

hipError_t launch_dd_final_reduce(const double* partials, int64_t np, double2* out_hi, double2* out_lo, double* abs_out,
                                  hipStream_t st) {
    hipLaunchKernelGGL(dd_final_reduce_kernel, dim3(1), dim3(64), 0, st, partials, np, out_hi, out_lo, abs_out);
    return hipGetLastError();
}

}  // namespace gbs
