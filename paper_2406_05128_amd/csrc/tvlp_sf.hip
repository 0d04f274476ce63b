// Source-filter synthesiser around the LP filter (Eq. 5): the pieces that wrap
// the chunked LP kernels.  Source u = p + C * n (frame-wise FIR filtering of
// the noise: each hop-sample frame of n is convolved with its own K taps and
// the results overlap-add), LP input x = gamma u with the gain gamma linearly
// upsampled from frame values (frame q at sample q*hop), and the trainable
// output FIR y = h * s.  float32 data, float32 accumulation of the products
// of one output (at most K), float64 where partial sums are combined.
//
// Layouts: signals [B][T]; C [B][F][K]; gain [B][F]; F = (T - 1) / hop + 2.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "tvlp.h"

namespace tvlp_sf {

constexpr int TT = 256;         // outputs per block of the convolution kernels
constexpr int KMAX = 1024;      // longest FIR
constexpr int HOPMAX = 4096;    // longest frame for the per-frame adjoint blocks

__device__ __forceinline__ float lerp_gain(const float *g, int64_t t, int hop) {
    const int64_t q = t / hop;
    const float w = (float)(t - q * hop) / (float)hop;
    return __builtin_fmaf(w, g[q + 1] - g[q], g[q]);
}

// u(t) = p(t) + sum_k C[q(t-k)][k] n(t-k), x(t) = gamma(t) u(t).  Block: TT
// consecutive outputs of one sequence; LDS holds n over [t0 - K + 1, t0 + TT).
// For an output t the taps are walked frame by frame (input samples tau from t
// down to t - K + 1), so the tap row of a stretch is fixed and lanes read
// consecutive taps.
__global__ __launch_bounds__(TT) void k_sf_source(int64_t T, int hop, int K, int64_t F, const float *__restrict__ p,
                                                  const float *__restrict__ n, const float *__restrict__ C,
                                                  const float *__restrict__ gain, float *__restrict__ u,
                                                  float *__restrict__ x) {
    extern __shared__ float ns[];  // TT + K - 1
    const int64_t b = blockIdx.y;
    const int64_t t0 = (int64_t)blockIdx.x * TT;
    const int64_t base = t0 - (K - 1);
    const float *nb = n + b * T;
    for (int i = threadIdx.x; i < TT + K - 1; i += TT) {
        const int64_t tau = base + i;
        ns[i] = (tau >= 0 && tau < T) ? nb[tau] : 0.f;
    }
    __syncthreads();
    const int64_t t = t0 + threadIdx.x;
    if (t >= T) return;
    const float *Cb = C + b * F * K;
    float acc = 0.f;
    const int64_t tau_min = t - (K - 1) > 0 ? t - (K - 1) : 0;
    int64_t hi = t;
    while (hi >= tau_min) {
        const int64_t q = hi / hop;
        const int64_t lo = q * hop > tau_min ? q * hop : tau_min;
        const float *Cq = Cb + q * K + (t - hi);  // tap k = t - tau
        const float *np_ = ns + (hi - base);
        const int cnt = (int)(hi - lo + 1);
        for (int j = 0; j < cnt; ++j) acc = __builtin_fmaf(Cq[j], np_[-j], acc);
        hi = lo - 1;
    }
    const float uu = p[b * T + t] + acc;
    u[b * T + t] = uu;
    x[b * T + t] = lerp_gain(gain + b * F, t, hop) * uu;
}

// y(t) = sum_k h[k] s(t-k) (corr = 0), or the adjoint in s,
// g_s(t) = sum_k h[k] g_y(t+k) (corr = 1).  LDS: the K taps, then the input over
// [t0 - K + 1, t0 + TT) (convolution) or [t0, t0 + TT + K - 1) (correlation).
__global__ __launch_bounds__(TT) void k_fir(int64_t T, int K, const float *__restrict__ in,
                                            const float *__restrict__ h, float *__restrict__ out, int corr) {
    extern __shared__ float sh[];
    float *hs = sh;
    float *xs = sh + K;
    const int64_t b = blockIdx.y;
    const int64_t t0 = (int64_t)blockIdx.x * TT;
    const int64_t base = corr ? t0 : t0 - (K - 1);
    const float *ib = in + b * T;
    for (int i = threadIdx.x; i < K; i += TT) hs[i] = h[i];
    for (int i = threadIdx.x; i < TT + K - 1; i += TT) {
        const int64_t tau = base + i;
        xs[i] = (tau >= 0 && tau < T) ? ib[tau] : 0.f;
    }
    __syncthreads();
    const int64_t t = t0 + threadIdx.x;
    if (t >= T) return;
    float acc0 = 0.f, acc1 = 0.f;
    const int li = threadIdx.x;
    if (corr) {
        int k = 0;
        for (; k + 1 < K; k += 2) {
            acc0 = __builtin_fmaf(hs[k], xs[li + k], acc0);
            acc1 = __builtin_fmaf(hs[k + 1], xs[li + k + 1], acc1);
        }
        if (k < K) acc0 = __builtin_fmaf(hs[k], xs[li + k], acc0);
    } else {
        const int c = li + K - 1;  // xs index of s(t)
        int k = 0;
        for (; k + 1 < K; k += 2) {
            acc0 = __builtin_fmaf(hs[k], xs[c - k], acc0);
            acc1 = __builtin_fmaf(hs[k + 1], xs[c - k - 1], acc1);
        }
        if (k < K) acc0 = __builtin_fmaf(hs[k], xs[c - k], acc0);
    }
    out[b * T + t] = acc0 + acc1;
}

constexpr int GT = 1024;  // samples per tile of the output-FIR gradient

// Partial dL/dh[k] = sum over one tile of sum_t g_y(t) s(t-k), per (sequence,
// tile); LDS: g_y over the tile, s over [t0 - K + 1, t0 + GT).
__global__ __launch_bounds__(256) void k_fir_gh_part(int64_t T, int K, const float *__restrict__ gy,
                                                     const float *__restrict__ s, float *__restrict__ part) {
    extern __shared__ float sh[];
    float *gs = sh;        // GT
    float *ss = sh + GT;   // GT + K - 1
    const int64_t b = blockIdx.y;
    const int64_t t0 = (int64_t)blockIdx.x * GT;
    for (int i = threadIdx.x; i < GT; i += blockDim.x) {
        const int64_t t = t0 + i;
        gs[i] = t < T ? gy[b * T + t] : 0.f;
    }
    for (int i = threadIdx.x; i < GT + K - 1; i += blockDim.x) {
        const int64_t tau = t0 - (K - 1) + i;
        ss[i] = (tau >= 0 && tau < T) ? s[b * T + tau] : 0.f;
    }
    __syncthreads();
    float *pb = part + ((int64_t)b * gridDim.x + blockIdx.x) * K;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        float acc0 = 0.f, acc1 = 0.f;
        const float *sk = ss + (K - 1 - k);  // sk[i] = s(t0 + i - k)
        for (int i = 0; i < GT; i += 2) {
            acc0 = __builtin_fmaf(gs[i], sk[i], acc0);
            acc1 = __builtin_fmaf(gs[i + 1], sk[i + 1], acc1);
        }
        pb[k] = acc0 + acc1;
    }
}

// dL/dh[k] = sum of the npart partials (float64, fixed order); one block per k.
__global__ __launch_bounds__(256) void k_sum_parts(int64_t npart, int K, const float *__restrict__ part,
                                                   float *__restrict__ out) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < npart; j += blockDim.x) acc += (double)part[j * K + k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = (float)red[0];
}

// g_u(t) = gamma(t) g_x(t) (also dL/dp), one thread per sample.
__global__ __launch_bounds__(256) void k_sf_gu(int64_t B, int64_t T, int hop, int64_t F,
                                               const float *__restrict__ gx, const float *__restrict__ gain,
                                               float *__restrict__ gu) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * T) return;
    const int64_t b = i / T, t = i - b * T;
    gu[i] = lerp_gain(gain + b * F, t, hop) * gx[i];
}

// One block per (frame q, sequence b):
//   dL/dC[q][k] = sum over the samples tau of frame q of g_u(tau + k) n(tau);
//   dL/dgain[q] = sum over frame q of (1 - w) g_x u + sum over frame q-1 of w g_x u,
//   w = (t - frame start) / hop.
// LDS: n over frame q, g_u over [q hop, q hop + hop + K - 1), g_x u over
// [(q-1) hop, (q+1) hop), a reduction buffer.
__global__ __launch_bounds__(256) void k_sf_frame_grads(int64_t T, int hop, int K, int64_t F,
                                                        const float *__restrict__ n, const float *__restrict__ gu,
                                                        const float *__restrict__ gx, const float *__restrict__ u,
                                                        float *__restrict__ gC, float *__restrict__ ggain) {
    extern __shared__ float sh[];
    __shared__ double red[256];
    const int64_t q = blockIdx.x, b = blockIdx.y;
    const int64_t lo = q * hop;
    float *ns = sh;                 // hop
    float *gus = ns + hop;          // hop + K - 1
    float *gxu = gus + hop + K - 1; // 2 hop, from (q-1) hop
    for (int i = threadIdx.x; i < hop; i += blockDim.x) {
        const int64_t t = lo + i;
        ns[i] = t < T ? n[b * T + t] : 0.f;
    }
    for (int i = threadIdx.x; i < hop + K - 1; i += blockDim.x) {
        const int64_t t = lo + i;
        gus[i] = t < T ? gu[b * T + t] : 0.f;
    }
    for (int i = threadIdx.x; i < 2 * hop; i += blockDim.x) {
        const int64_t t = lo - hop + i;
        gxu[i] = (t >= 0 && t < T) ? gx[b * T + t] * u[b * T + t] : 0.f;
    }
    __syncthreads();
    // the frame's taps (frames at or beyond the signal's end get zeros)
    float *gCq = gC + (b * F + q) * K;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        float acc0 = 0.f, acc1 = 0.f;
        int i = 0;
        for (; i + 1 < hop; i += 2) {
            acc0 = __builtin_fmaf(gus[i + k], ns[i], acc0);
            acc1 = __builtin_fmaf(gus[i + k + 1], ns[i + 1], acc1);
        }
        if (i < hop) acc0 = __builtin_fmaf(gus[i + k], ns[i], acc0);
        gCq[k] = acc0 + acc1;
    }
    // the frame's gain
    double acc = 0.0;
    for (int i = threadIdx.x; i < 2 * hop; i += blockDim.x) {
        const int nn = i < hop ? i : i - hop;
        const double w = (double)nn / hop;
        acc += (i < hop ? w : 1.0 - w) * (double)gxu[i];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) ggain[b * F + q] = (float)red[0];
}

thread_local char g_msg[256];

int fail(int code, const char *msg) {
    snprintf(g_msg, sizeof g_msg, "%s", msg);
    return code;
}

int launched(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return LP_OK;
    snprintf(g_msg, sizeof g_msg, "%s: %s", what, hipGetErrorString(e));
    return LP_EDEVICE;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace tvlp_sf

using namespace tvlp_sf;

extern "C" {

const char *lp_sf_last_error(void) { return g_msg; }

int lp_sf_source(int64_t B, int64_t T, int64_t hop, int64_t K, const float *p, const float *n, const float *C,
                 const float *gain, float *u, float *x, void *stream) {
    if (B < 1 || T < 1 || hop < 1 || hop > HOPMAX || K < 1 || K > KMAX)
        return fail(LP_EINVAL, "lp_sf_source: need B, T >= 1, 1 <= hop <= 4096, 1 <= K <= 1024");
    if (!p || !n || !C || !gain || !u || !x) return fail(LP_EINVAL, "lp_sf_source: null pointer");
    if (B > 65535) return fail(LP_EINVAL, "lp_sf_source: B > 65535");
    const int64_t F = (T - 1) / hop + 2;
    hipLaunchKernelGGL(k_sf_source, dim3((unsigned)ceil_div(T, TT), (unsigned)B), dim3(TT),
                       (size_t)(TT + K - 1) * sizeof(float), (hipStream_t)stream, T, (int)hop, (int)K, F, p, n, C,
                       gain, u, x);
    return launched("lp_sf_source");
}

int lp_fir(int64_t B, int64_t T, int64_t K, const float *s, const float *h, float *y, void *stream) {
    if (B < 1 || T < 1 || K < 1 || K > KMAX || B > 65535)
        return fail(LP_EINVAL, "lp_fir: need B in [1, 65535], T >= 1, 1 <= K <= 1024");
    if (!s || !h || !y) return fail(LP_EINVAL, "lp_fir: null pointer");
    hipLaunchKernelGGL(k_fir, dim3((unsigned)ceil_div(T, TT), (unsigned)B), dim3(TT),
                       (size_t)(TT + 2 * K - 1) * sizeof(float), (hipStream_t)stream, T, (int)K, s, h, y, 0);
    return launched("lp_fir");
}

size_t lp_fir_adjoint_work_bytes(int64_t B, int64_t T, int64_t K) {
    if (B < 1 || T < 1 || K < 1) return 0;
    return (size_t)B * ceil_div(T, GT) * K * sizeof(float);
}

int lp_fir_adjoint(int64_t B, int64_t T, int64_t K, const float *gy, const float *s, const float *h, float *gs,
                   float *gh, void *work, void *stream) {
    if (B < 1 || T < 1 || K < 1 || K > KMAX || B > 65535)
        return fail(LP_EINVAL, "lp_fir_adjoint: need B in [1, 65535], T >= 1, 1 <= K <= 1024");
    if (!gy || !h || (gh && (!s || !work))) return fail(LP_EINVAL, "lp_fir_adjoint: null pointer");
    hipStream_t st = (hipStream_t)stream;
    if (gs)
        hipLaunchKernelGGL(k_fir, dim3((unsigned)ceil_div(T, TT), (unsigned)B), dim3(TT),
                           (size_t)(TT + 2 * K - 1) * sizeof(float), st, T, (int)K, gy, h, gs, 1);
    if (gh) {
        const int64_t nt = ceil_div(T, GT);
        float *part = (float *)work;
        hipLaunchKernelGGL(k_fir_gh_part, dim3((unsigned)nt, (unsigned)B), dim3(256),
                           (size_t)(2 * GT + K - 1) * sizeof(float), st, T, (int)K, gy, s, part);
        hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)K), dim3(256), 0, st, B * nt, (int)K, part, gh);
    }
    return launched("lp_fir_adjoint");
}

int lp_sf_source_adjoint(int64_t B, int64_t T, int64_t hop, int64_t K, const float *gx, const float *u,
                         const float *n, const float *gain, float *gu, float *gC, float *ggain, void *stream) {
    if (B < 1 || T < 1 || hop < 1 || hop > HOPMAX || K < 1 || K > KMAX || B > 65535)
        return fail(LP_EINVAL, "lp_sf_source_adjoint: need B in [1, 65535], T >= 1, 1 <= hop <= 4096, 1 <= K <= 1024");
    if (!gx || !u || !n || !gain || !gu || !gC || !ggain) return fail(LP_EINVAL, "lp_sf_source_adjoint: null pointer");
    hipStream_t st = (hipStream_t)stream;
    const int64_t F = (T - 1) / hop + 2;
    hipLaunchKernelGGL(k_sf_gu, dim3((unsigned)ceil_div(B * T, 256)), dim3(256), 0, st, B, T, (int)hop, F, gx, gain,
                       gu);
    hipLaunchKernelGGL(k_sf_frame_grads, dim3((unsigned)F, (unsigned)B), dim3(256),
                       (size_t)(4 * hop + K - 1) * sizeof(float), st, T, (int)hop, (int)K, F, n, gu, gx, u, gC,
                       ggain);
    return launched("lp_sf_source_adjoint");
}

}  // extern "C"
