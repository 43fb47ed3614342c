// Kernels of the conditional sampling chain (Sec. III of the paper): the
// heterodyne outcomes of modes 2..M, the per-step loop-hafnian matrices of the
// conditional pure states, and the photon-number draws.  The loop hafnians
// themselves run through the batch kernels.
#include <hip/hip_runtime.h>

#include "lhaf_kernels.h"

namespace gbs {

namespace {

constexpr int kBuildThreads = 256;

// x = mean + L z per sample (L lower triangular, dim x dim, row-major); the
// complex outcome of mode i is x[i] + i x[h + i], h = dim / 2.
__global__ void __launch_bounds__(64) heterodyne_kernel(const double* __restrict__ L, const double* __restrict__ mean,
                                                        int dim, const double* __restrict__ normals,
                                                        double2* __restrict__ beta) {
    const int b = blockIdx.x;
    const double* z = normals + (int64_t)b * dim;
    const int h = dim / 2;
    for (int i = threadIdx.x; i < h; i += blockDim.x) {
        double re = mean[i], im = mean[h + i];
        const double* lr = L + (int64_t)i * dim;
        const double* li = L + (int64_t)(h + i) * dim;
        for (int t = 0; t <= i; ++t) re = fma(lr[t], z[t], re);
        for (int t = 0; t <= h + i; ++t) im = fma(li[t], z[t], im);
        beta[(int64_t)b * h + i] = make_double2(re, im);
    }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// One block per sample: loop weights gamma = c + F [beta_B; conj(beta_B)] of
// the conditional state of modes 1..k, then the cutoff + 1 matrices
// filldiag(B_S, gamma_S) of the patterns (s_1, .., s_{k-1}, j), j = 0..cutoff.
__global__ void __launch_bounds__(kBuildThreads) sampler_build_kernel(SamplerStep p) {
    __shared__ double2 gam[kMaxSamplerModes];
    __shared__ int idx[2 * kMaxPairs + 1];
    __shared__ int prefix;
    const int b = blockIdx.x;
    const int k = p.k, nb = p.M - k;  // conditioned modes k+1..M (1-based)
    const double2* beta = p.beta + (int64_t)b * (p.M - 1) + (k - 1);
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        double2 g = p.ck[i];
        const double2* f = p.Fk + (int64_t)i * 2 * nb;
        for (int t = 0; t < nb; ++t) {
            const double2 bt = beta[t];
            const double2 a = cmul(f[t], bt);
            const double2 c = cmul(f[nb + t], make_double2(bt.x, -bt.y));
            g.x += a.x + c.x;
            g.y += a.y + c.y;
        }
        gam[i] = g;
    }
    if (threadIdx.x == 0) {
        // row/column u of the expanded matrix belongs to mode idx[u]
        int u = 0;
        for (int i = 0; i + 1 < k; ++i) {
            const int s = p.samples[(int64_t)i * p.nsamples + b];
            for (int c = 0; c < s && u < 2 * kMaxPairs; ++c) idx[u++] = i;
        }
        prefix = u;
        for (int c = 0; c < p.cutoff && u < 2 * kMaxPairs + 1; ++c) idx[u++] = k - 1;
    }
    __syncthreads();
    const int P = prefix;
    for (int j = 0; j <= p.cutoff; ++j) {
        const int64_t item = (int64_t)b * (p.cutoff + 1) + j;
        const int N = p.dims[item];
        if (N != P + j || N > 2 * kMaxPairs) continue;  // the host sized the item from the same draws
        double2* out = p.mats + p.in_off[item];
        for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
            const int u = e / N, v = e - u * N;
            out[e] = (u == v) ? gam[idx[u]] : p.Bk[idx[u] * k + idx[v]];
        }
    }
}

// One lane per sample: w_j = |lhaf_j|^2 / j!, normalised over j = 0..cutoff,
// and the draw s = #{j : cdf_j <= u} (at most cutoff).  -1 marks weights that
// are not finite or sum to zero.
__global__ void __launch_bounds__(64) sampler_draw_kernel(const double2* __restrict__ lh, int nsamples, int cutoff,
                                                          const double* __restrict__ u, int* __restrict__ draw,
                                                          double* __restrict__ probs, int64_t probs_stride) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nsamples) return;
    const double2* l = lh + (int64_t)b * (cutoff + 1);
    // two passes (sum, then cdf) so that no per-lane array is needed
    double W = 0.0, fact = 1.0;
    for (int j = 0; j <= cutoff; ++j) {
        if (j > 1) fact *= (double)j;
        W += (l[j].x * l[j].x + l[j].y * l[j].y) / fact;
    }
    if (!(W > 0.0) || !(W < INFINITY)) {
        draw[b] = -1;
        return;
    }
    const double ub = u[b];
    double cdf = 0.0;
    int s = 0;
    fact = 1.0;
    for (int j = 0; j <= cutoff; ++j) {
        if (j > 1) fact *= (double)j;
        const double pj = ((l[j].x * l[j].x + l[j].y * l[j].y) / fact) / W;
        if (probs) probs[(int64_t)b * probs_stride + j] = pj;
        cdf += pj;
        if (cdf <= ub) s = j + 1;
    }
    draw[b] = s < cutoff ? s : cutoff;
}

}  // namespace

hipError_t launch_heterodyne(const double* L, const double* mean, int dim, const double* normals, int nsamples,
                             double2* beta, hipStream_t st) {
    if (nsamples <= 0 || dim <= 0) return hipSuccess;
    hipLaunchKernelGGL(heterodyne_kernel, dim3(nsamples), dim3(64), 0, st, L, mean, dim, normals, beta);
    return hipGetLastError();
}

hipError_t launch_sampler_build(const SamplerStep& p, hipStream_t st) {
    if (p.nsamples <= 0) return hipSuccess;
    if (p.k < 1 || p.k > p.M || p.M > kMaxSamplerModes || p.cutoff < 0 || p.cutoff > kMaxCutoff)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(sampler_build_kernel, dim3(p.nsamples), dim3(kBuildThreads), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_sampler_draw(const double2* lh, int nsamples, int cutoff, const double* u, int* draw, double* probs,
                               int64_t probs_stride, hipStream_t st) {
    if (nsamples <= 0) return hipSuccess;
    if (cutoff < 0 || cutoff > kMaxCutoff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sampler_draw_kernel, dim3((nsamples + 63) / 64), dim3(64), 0, st, lh, nsamples, cutoff, u, draw,
                       probs, probs_stride);
    return hipGetLastError();
}

}  // namespace gbs
