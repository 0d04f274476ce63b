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

// The same source, register-blocked: a block of SW_WAVES waves covers
// SW_WAVES * TT consecutive outputs, each wave TT of them, RB per lane (lane j:
// t_j = t0 + RB j .. + RB - 1); the frame rows of taps the block reads are
// staged in LDS once, with PAD zeros on either side, so that each wave walks the
// input samples tau of its tile in lockstep (taps outside a row read zeros).  Each lane keeps the window of RB taps C[q][t_j + r - tau]; when
// tau advances, the tap entering lane j's window is the one leaving lane j-1's,
// so it moves one lane up by a wave-wide DPP shift, lane 0 taking it from a
// broadcast read of the row.  Per tau: two broadcast LDS reads (n and lane 0's
// tap), one DPP move and RB FMAs.
constexpr int RB = 4;
constexpr int PAD = TT + 2 * RB;
constexpr int SW_WAVES = 4;
constexpr int DPP_WAVE_SHR1 = 0x138;  // lane i <- lane i-1 across the wave (lane 0 keeps `old`)
constexpr int DPP_WAVE_SHL1 = 0x130;  // lane i <- lane i+1 across the wave (lane 63 keeps `old`)

template <int CTRL>
__device__ __forceinline__ float wave_shift(float v, float old) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, 0xF, 0xF, false));
}

__global__ __launch_bounds__(64 * SW_WAVES) void k_sf_source_rb(int64_t T, int hop, int K, int64_t F,
                                                                const float *__restrict__ p,
                                                                const float *__restrict__ n,
                                                                const float *__restrict__ C,
                                                                const float *__restrict__ gain,
                                                                float *__restrict__ u, float *__restrict__ x) {
    extern __shared__ float sh[];
    constexpr int BT = SW_WAVES * TT;  // outputs per block
    const int SW = K + 2 * PAD;        // staged row width
    const int64_t b = blockIdx.y;
    const int64_t t0b = (int64_t)blockIdx.x * BT;
    const int64_t tlo = t0b - (K - 1);                              // first input sample of the block
    const int64_t qlo = (tlo > 0 ? tlo : 0) / hop;
    const int64_t tlast = t0b + BT - 1 < T - 1 ? t0b + BT - 1 : T - 1;
    const int nrow = (int)(tlast / hop - qlo + 1);
    float *ns = sh;                  // n(tau) at tau - tlo, BT + K - 1 floats
    float *rows = sh + BT + K - 1;   // staged rows, nrow x SW
    const float *nb = n + b * T;
    for (int i = threadIdx.x; i < BT + K - 1; i += 64 * SW_WAVES) {
        const int64_t tau = tlo + i;
        ns[i] = (tau >= 0 && tau < T) ? nb[tau] : 0.f;
    }
    for (int r = 0; r < nrow; ++r) {
        const float *Cq = C + (b * F + qlo + r) * K;
        float *row = rows + r * SW;
        for (int i = threadIdx.x; i < SW; i += 64 * SW_WAVES) {
            const int k = i - PAD;
            row[i] = (k >= 0 && k < K) ? Cq[k] : 0.f;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    // the wave index is uniform in the wave; saying so keeps the tile walk's
    // counters and addresses in scalar registers
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = t0b + (int64_t)TT * wv;     // this wave's tile
    if (t0 >= T) return;
    const int64_t ta = t0 - (K - 1) > 0 ? t0 - (K - 1) : 0;         // the tile's first input sample
    const int64_t tb = t0 + TT - 1 < T - 1 ? t0 + TT - 1 : T - 1;   // and last
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    int64_t tau = ta;
    while (tau <= tb) {
        const int64_t q = tau / hop;
        const int64_t end = (q + 1) * hop - 1 < tb ? (q + 1) * hop - 1 : tb;  // last tau of this frame's stretch
        const float *row = rows + (q - qlo) * SW;
        int b0 = (int)(PAD + t0 - tau);  // row index of lane 0's tap t0 - tau
        const int bi = b0 + RB * lane;   // this lane's
        float w0 = row[bi], w1 = row[bi + 1], w2 = row[bi + 2], w3 = row[bi + 3];
        const float *nt = ns + (tau - tlo);
        int cnt = (int)(end - tau + 1);
        // Four steps: each window register is shifted in place right after its
        // last use at the current offset (w3 after the first step, w2 after the
        // second, ...), so after the four steps w0..w3 already hold the window
        // four samples on.  A DPP move's result cannot share its source register,
        // so the loop runs two such blocks per pass, letting the two register
        // sets alternate without copies.
        auto step4 = [&]() {
            float v = nt[0];
            a0 = __builtin_fmaf(w0, v, a0); a1 = __builtin_fmaf(w1, v, a1);
            a2 = __builtin_fmaf(w2, v, a2); a3 = __builtin_fmaf(w3, v, a3);
            w3 = wave_shift<DPP_WAVE_SHR1>(w3, row[b0 - 1]);
            v = nt[1];
            a0 = __builtin_fmaf(w3, v, a0); a1 = __builtin_fmaf(w0, v, a1);
            a2 = __builtin_fmaf(w1, v, a2); a3 = __builtin_fmaf(w2, v, a3);
            w2 = wave_shift<DPP_WAVE_SHR1>(w2, row[b0 - 2]);
            v = nt[2];
            a0 = __builtin_fmaf(w2, v, a0); a1 = __builtin_fmaf(w3, v, a1);
            a2 = __builtin_fmaf(w0, v, a2); a3 = __builtin_fmaf(w1, v, a3);
            w1 = wave_shift<DPP_WAVE_SHR1>(w1, row[b0 - 3]);
            v = nt[3];
            a0 = __builtin_fmaf(w1, v, a0); a1 = __builtin_fmaf(w2, v, a1);
            a2 = __builtin_fmaf(w3, v, a2); a3 = __builtin_fmaf(w0, v, a3);
            w0 = wave_shift<DPP_WAVE_SHR1>(w0, row[b0 - 4]);
            b0 -= 4;
            nt += 4;
            cnt -= 4;
        };
        while (cnt >= 8) {
            step4();
            step4();
        }
        if (cnt >= 4) step4();
        while (cnt > 0) {
            const float x1 = wave_shift<DPP_WAVE_SHR1>(w3, row[b0 - 1]);
            const float v = nt[0];
            a0 = __builtin_fmaf(w0, v, a0); a1 = __builtin_fmaf(w1, v, a1);
            a2 = __builtin_fmaf(w2, v, a2); a3 = __builtin_fmaf(w3, v, a3);
            w3 = w2; w2 = w1; w1 = w0; w0 = x1;
            b0 -= 1;
            nt += 1;
            cnt -= 1;
        }
        tau = end + 1;
    }
    const float acc[RB] = {a0, a1, a2, a3};
    const float *gb = gain + b * F;
    const int64_t tj = t0 + RB * lane;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int64_t t = tj + r;
        if (t < T) {
            const float uu = p[b * T + t] + acc[r];
            u[b * T + t] = uu;
            x[b * T + t] = lerp_gain(gb, t, hop) * uu;
        }
    }
}

// Staged-row bytes of k_sf_source_rb for the worst block (0: the rows do not fit).
size_t source_rb_lds(int hop, int K) {
    const int64_t span = SW_WAVES * TT + K - 1;
    const int64_t nrow = (span - 1) / hop + 2;
    const size_t bytes = (size_t)(span + nrow * (K + 2 * PAD)) * sizeof(float);
    return bytes <= 128 * 1024 ? bytes : 0;
}

// The output FIR register-blocked: a block of SW_WAVES waves covers
// SW_WAVES * TT outputs, RB per lane (lane j: t_j = t0 + RB j ..); per tap k every
// lane updates its RB outputs from a window of RB input samples, which slides by
// one sample per tap: the entering sample is the one leaving the neighbouring
// lane's window (wave-wide DPP shift; the edge lane reads it from LDS).
// Convolution (CORR = false): y(t) = sum_k h[k] s(t - k), window s(t_j + r - k),
// entering from lane j-1.  Correlation (CORR = true): g_s(t) = sum_k h[k] g_y(t + k),
// window g_y(t_j + r + k), entering from lane j+1.  LDS: the K taps, then the
// input over [t0 - K + 1, t0 + BT) or [t0, t0 + BT + K - 1), zeros outside the
// signal, plus RB floats of slack.
template <bool CORR>
__global__ __launch_bounds__(64 * SW_WAVES) void k_fir_rb(int64_t T, int K, const float *__restrict__ in,
                                                          const float *__restrict__ h, float *__restrict__ out) {
    extern __shared__ float sh[];
    constexpr int BT = SW_WAVES * TT;
    float *hs = sh;
    float *xs = sh + K;
    const int64_t b = blockIdx.y;
    const int64_t t0b = (int64_t)blockIdx.x * BT;
    const int64_t base = CORR ? t0b : t0b - (K - 1);  // input sample of xs[0]
    const float *ib = in + b * T;
    for (int i = threadIdx.x; i < K; i += 64 * SW_WAVES) hs[i] = h[i];
    for (int i = threadIdx.x; i < BT + K - 1 + RB; i += 64 * SW_WAVES) {
        const int64_t tau = base + i;
        xs[i] = (tau >= 0 && tau < T) ? ib[tau] : 0.f;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t t0 = t0b + (int64_t)TT * (threadIdx.x >> 6);
    if (t0 >= T) return;
    const int o0 = (int)(t0 - base);  // xs index of input sample t0 (convolution) / t0 (correlation)
    const int oj = o0 + RB * lane;    // this lane's t_j
    float w0 = xs[oj], w1 = xs[oj + 1], w2 = xs[oj + 2], w3 = xs[oj + 3];  // window at k = 0
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    // Four taps per block with each window register shifted in place after its
    // last use, two blocks per pass (the DPP results alternate between two
    // register sets); the remaining taps take the one-tap step below.
    auto block4 = [&](int k) {
        float h = hs[k];
        a0 = __builtin_fmaf(h, w0, a0); a1 = __builtin_fmaf(h, w1, a1);
        a2 = __builtin_fmaf(h, w2, a2); a3 = __builtin_fmaf(h, w3, a3);
        if constexpr (CORR) {
            w0 = wave_shift<DPP_WAVE_SHL1>(w0, xs[o0 + 256 + k]);
            h = hs[k + 1];
            a0 = __builtin_fmaf(h, w1, a0); a1 = __builtin_fmaf(h, w2, a1);
            a2 = __builtin_fmaf(h, w3, a2); a3 = __builtin_fmaf(h, w0, a3);
            w1 = wave_shift<DPP_WAVE_SHL1>(w1, xs[o0 + 256 + k + 1]);
            h = hs[k + 2];
            a0 = __builtin_fmaf(h, w2, a0); a1 = __builtin_fmaf(h, w3, a1);
            a2 = __builtin_fmaf(h, w0, a2); a3 = __builtin_fmaf(h, w1, a3);
            w2 = wave_shift<DPP_WAVE_SHL1>(w2, xs[o0 + 256 + k + 2]);
            h = hs[k + 3];
            a0 = __builtin_fmaf(h, w3, a0); a1 = __builtin_fmaf(h, w0, a1);
            a2 = __builtin_fmaf(h, w1, a2); a3 = __builtin_fmaf(h, w2, a3);
            w3 = wave_shift<DPP_WAVE_SHL1>(w3, xs[o0 + 256 + k + 3]);
        } else {
            w3 = wave_shift<DPP_WAVE_SHR1>(w3, xs[o0 - 1 - k]);
            h = hs[k + 1];
            a0 = __builtin_fmaf(h, w3, a0); a1 = __builtin_fmaf(h, w0, a1);
            a2 = __builtin_fmaf(h, w1, a2); a3 = __builtin_fmaf(h, w2, a3);
            w2 = wave_shift<DPP_WAVE_SHR1>(w2, xs[o0 - 2 - k]);
            h = hs[k + 2];
            a0 = __builtin_fmaf(h, w2, a0); a1 = __builtin_fmaf(h, w3, a1);
            a2 = __builtin_fmaf(h, w0, a2); a3 = __builtin_fmaf(h, w1, a3);
            w1 = wave_shift<DPP_WAVE_SHR1>(w1, xs[o0 - 3 - k]);
            h = hs[k + 3];
            a0 = __builtin_fmaf(h, w1, a0); a1 = __builtin_fmaf(h, w2, a1);
            a2 = __builtin_fmaf(h, w3, a2); a3 = __builtin_fmaf(h, w0, a3);
            w0 = wave_shift<DPP_WAVE_SHR1>(w0, xs[o0 - 4 - k]);
        }
    };
    int k = 0;
    for (; k + 8 <= K; k += 8) {
        block4(k);
        block4(k + 4);
    }
    if (k + 4 <= K) {
        block4(k);
        k += 4;
    }
    for (; k < K; ++k) {
        const float hk = hs[k];
        a0 = __builtin_fmaf(hk, w0, a0); a1 = __builtin_fmaf(hk, w1, a1);
        a2 = __builtin_fmaf(hk, w2, a2); a3 = __builtin_fmaf(hk, w3, a3);
        if constexpr (CORR) {
            // next window g_y(t_j + r + k + 1): w0..w2 <- w1..w3, w3 <- lane j+1's w0
            const float e = wave_shift<DPP_WAVE_SHL1>(w0, xs[o0 + 256 + k]);
            w0 = w1; w1 = w2; w2 = w3; w3 = e;
        } else {
            // next window s(t_j + r - k - 1): w1..w3 <- w0..w2, w0 <- lane j-1's w3
            const float e = wave_shift<DPP_WAVE_SHR1>(w3, xs[o0 - 1 - k]);
            w3 = w2; w2 = w1; w1 = w0; w0 = e;
        }
    }
    const float acc[RB] = {a0, a1, a2, a3};
    const int64_t tj = t0 + RB * lane;
#pragma unroll
    for (int r = 0; r < RB; ++r)
        if (tj + r < T) out[b * T + tj + r] = acc[r];
}

constexpr int GT = 1024;  // samples per tile of the output-FIR gradient

// Partial dL/dh[k] = sum_t g_y(t) s(t-k) over one tile, per (sequence, tile):
// wave w of the block takes samples t0 + 256 w .. + 255 and the four waves'
// sums are added in LDS.
// Lane j owns taps k = 64 RT g + RT j + r (r < RT) of tap group g and keeps the
// window s(t - k); when t advances, the element entering lane j's window is the
// one leaving lane j-1's (wave-wide DPP shift; lane 0 reads it from LDS).
// LDS: g_y over the tile, s over [t0 - K + 1, t0 + GT] (zeros outside the signal;
// the last element is only read as the window's unused look-ahead), then the
// waves' sums [4][K].
template <int RT>
__global__ __launch_bounds__(256) void k_fir_gh_part(int64_t T, int K, const float *__restrict__ gy,
                                                     const float *__restrict__ s, float *__restrict__ part) {
    extern __shared__ float sh[];
    float *gs = sh;        // GT
    float *ss = sh + GT;   // GT + K
    float *wsum = ss + GT + K;  // 4 x K
    const int64_t b = blockIdx.y;
    const int64_t t0 = (int64_t)blockIdx.x * GT;
    for (int i = threadIdx.x; i < GT; i += blockDim.x) {
        const int64_t t = t0 + i;
        gs[i] = t < T ? gy[b * T + t] : 0.f;
    }
    for (int i = threadIdx.x; i < GT + K; i += blockDim.x) {
        const int64_t tau = t0 - (K - 1) + i;
        ss[i] = (tau >= 0 && tau < T) ? s[b * T + tau] : 0.f;
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i0 = 256 * wv;  // the wave's first sample in the tile
    for (int kg = 0; kg < K; kg += 64 * RT) {
        const int k0 = kg + RT * lane;
        // ss index of s(t0 + i - k) is i - k + K - 1
        float w[RT], acc[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const int k = k0 + r;
            w[r] = k < K ? ss[i0 - k + K - 1] : 0.f;
            acc[r] = 0.f;
        }
        for (int i = i0; i < i0 + 256; ++i) {
            const float gv = gs[i];
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = __builtin_fmaf(gv, w[r], acc[r]);
            // next window s(t0 + i + 1 - k): w[r] <- w[r-1], w[0] <- lane j-1's w[RT-1]
            const float e = wave_shift<DPP_WAVE_SHR1>(w[RT - 1], ss[i + 1 - kg + K - 1]);
#pragma unroll
            for (int r = RT - 1; r > 0; --r) w[r] = w[r - 1];
            w[0] = e;
        }
#pragma unroll
        for (int r = 0; r < RT; ++r)
            if (k0 + r < K) wsum[wv * K + k0 + r] = acc[r];
    }
    __syncthreads();
    float *pb = part + ((int64_t)b * gridDim.x + blockIdx.x) * K;
    for (int k = threadIdx.x; k < K; k += blockDim.x)
        pb[k] = (wsum[k] + wsum[K + k]) + (wsum[2 * K + k] + wsum[3 * K + k]);
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
// Taps: wave w, lane j owns k = 256 w + RB j + r (r < RB) and keeps the window
// g_u(tau + k); when tau advances the element entering lane j's window is the
// one leaving lane j+1's (a wave-wide DPP shift down; lane 63 reads it from
// LDS).  LDS: n over frame q, g_u over [q hop, q hop + hop + GUW) (zeros
// beyond the signal), g_x u over [(q-1) hop, (q+1) hop), a reduction buffer.
constexpr int GUW = KMAX + 16;
__global__ __launch_bounds__(256) void k_sf_frame_grads(int64_t T, int hop, int K, int64_t F,
                                                        const float *__restrict__ n, const float *__restrict__ gu,
                                                        const float *__restrict__ gx, const float *__restrict__ u,
                                                        float *__restrict__ gC, float *__restrict__ ggain) {
    extern __shared__ float sh[];
    __shared__ double red[256];
    const int64_t q = blockIdx.x, b = blockIdx.y;
    const int64_t lo = q * hop;
    float *ns = sh;                  // hop
    float *gus = ns + hop;           // hop + GUW
    float *gxu = gus + hop + GUW;    // 2 hop, from (q-1) hop
    for (int i = threadIdx.x; i < hop; i += blockDim.x) {
        const int64_t t = lo + i;
        ns[i] = t < T ? n[b * T + t] : 0.f;
    }
    for (int i = threadIdx.x; i < hop + GUW; i += blockDim.x) {
        const int64_t t = lo + i;
        gus[i] = (i < hop + K - 1 && t < T) ? gu[b * T + t] : 0.f;
    }
    for (int i = threadIdx.x; i < 2 * hop; i += blockDim.x) {
        const int64_t t = lo - hop + i;
        gxu[i] = (t >= 0 && t < T) ? gx[b * T + t] * u[b * T + t] : 0.f;
    }
    __syncthreads();
    // the frame's taps (frames at or beyond the signal's end get zeros)
    {
        const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
        const int kw = 256 * wv;                   // the wave's first tap
        const int k0 = kw + RB * lane;             // this lane's first tap
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
        float w0 = gus[k0], w1 = gus[k0 + 1], w2 = gus[k0 + 2], w3 = gus[k0 + 3];
        const float *g63 = gus + kw + 256;  // lane 63's entering elements: g63[i + s - 1] at step i + s
        int i = 0;
        // Four steps with each window register shifted in place after its last
        // use (w0 after the first step, w1 after the second, ...), two blocks
        // per pass so that the DPP results alternate between two register sets.
        auto step4 = [&](int i4) {
            float v = ns[i4];
            a0 = __builtin_fmaf(w0, v, a0); a1 = __builtin_fmaf(w1, v, a1);
            a2 = __builtin_fmaf(w2, v, a2); a3 = __builtin_fmaf(w3, v, a3);
            w0 = wave_shift<DPP_WAVE_SHL1>(w0, g63[i4]);
            v = ns[i4 + 1];
            a0 = __builtin_fmaf(w1, v, a0); a1 = __builtin_fmaf(w2, v, a1);
            a2 = __builtin_fmaf(w3, v, a2); a3 = __builtin_fmaf(w0, v, a3);
            w1 = wave_shift<DPP_WAVE_SHL1>(w1, g63[i4 + 1]);
            v = ns[i4 + 2];
            a0 = __builtin_fmaf(w2, v, a0); a1 = __builtin_fmaf(w3, v, a1);
            a2 = __builtin_fmaf(w0, v, a2); a3 = __builtin_fmaf(w1, v, a3);
            w2 = wave_shift<DPP_WAVE_SHL1>(w2, g63[i4 + 2]);
            v = ns[i4 + 3];
            a0 = __builtin_fmaf(w3, v, a0); a1 = __builtin_fmaf(w0, v, a1);
            a2 = __builtin_fmaf(w1, v, a2); a3 = __builtin_fmaf(w2, v, a3);
            w3 = wave_shift<DPP_WAVE_SHL1>(w3, g63[i4 + 3]);
        };
        for (; i + 8 <= hop; i += 8) {
            step4(i);
            step4(i + 4);
        }
        if (i + 4 <= hop) {
            step4(i);
            i += 4;
        }
        for (; i < hop; ++i) {
            const float y1 = wave_shift<DPP_WAVE_SHL1>(w0, g63[i]);
            const float v = ns[i];
            a0 = __builtin_fmaf(w0, v, a0); a1 = __builtin_fmaf(w1, v, a1);
            a2 = __builtin_fmaf(w2, v, a2); a3 = __builtin_fmaf(w3, v, a3);
            w0 = w1; w1 = w2; w2 = w3; w3 = y1;
        }
        float *gCq = gC + (b * F + q) * K;
        const float acc[RB] = {a0, a1, a2, a3};
#pragma unroll
        for (int r = 0; r < RB; ++r)
            if (k0 + r < K) gCq[k0 + r] = acc[r];
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
    if (const size_t lds = source_rb_lds((int)hop, (int)K))
        hipLaunchKernelGGL(k_sf_source_rb, dim3((unsigned)ceil_div(T, SW_WAVES * TT), (unsigned)B),
                           dim3(64 * SW_WAVES), lds, (hipStream_t)stream, T, (int)hop, (int)K, F, p, n, C, gain, u,
                           x);
    else  // short frames: too many tap rows per tile to stage
        hipLaunchKernelGGL(k_sf_source, dim3((unsigned)ceil_div(T, TT), (unsigned)B), dim3(TT),
                           (size_t)(TT + K - 1) * sizeof(float), (hipStream_t)stream, T, (int)hop, (int)K, F, p, n,
                           C, gain, u, x);
    return launched("lp_sf_source");
}

int lp_fir(int64_t B, int64_t T, int64_t K, const float *s, const float *h, float *y, void *stream) {
    if (B < 1 || T < 1 || K < 1 || K > KMAX || B > 65535)
        return fail(LP_EINVAL, "lp_fir: need B in [1, 65535], T >= 1, 1 <= K <= 1024");
    if (!s || !h || !y) return fail(LP_EINVAL, "lp_fir: null pointer");
    hipLaunchKernelGGL(k_fir_rb<false>, dim3((unsigned)ceil_div(T, SW_WAVES * TT), (unsigned)B),
                       dim3(64 * SW_WAVES), (size_t)(SW_WAVES * TT + 2 * K - 1 + RB) * sizeof(float),
                       (hipStream_t)stream, T, (int)K, s, h, y);
    return launched("lp_fir");
}

size_t lp_fir_adjoint_work_bytes(int64_t B, int64_t T, int64_t K) {
    if (B < 1 || T < 1 || K < 1) return 0;
    return (size_t)B * ceil_div(T, GT) * K * sizeof(float);  // one partial row per tile
}

int lp_fir_adjoint(int64_t B, int64_t T, int64_t K, const float *gy, const float *s, const float *h, float *gs,
                   float *gh, void *work, void *stream) {
    if (B < 1 || T < 1 || K < 1 || K > KMAX || B > 65535)
        return fail(LP_EINVAL, "lp_fir_adjoint: need B in [1, 65535], T >= 1, 1 <= K <= 1024");
    if (!gy || !h || (gh && (!s || !work))) return fail(LP_EINVAL, "lp_fir_adjoint: null pointer");
    hipStream_t st = (hipStream_t)stream;
    if (gs)
        hipLaunchKernelGGL(k_fir_rb<true>, dim3((unsigned)ceil_div(T, SW_WAVES * TT), (unsigned)B),
                           dim3(64 * SW_WAVES), (size_t)(SW_WAVES * TT + 2 * K - 1 + RB) * sizeof(float), st, T,
                           (int)K, gy, h, gs);
    if (gh) {
        const int64_t nt = ceil_div(T, GT);
        float *part = (float *)work;
        const size_t lds = (size_t)(2 * GT + 5 * K) * sizeof(float);
        if (K <= 128)
            hipLaunchKernelGGL(k_fir_gh_part<2>, dim3((unsigned)nt, (unsigned)B), dim3(256), lds, st, T, (int)K, gy,
                               s, part);
        else
            hipLaunchKernelGGL(k_fir_gh_part<4>, dim3((unsigned)nt, (unsigned)B), dim3(256), lds, st, T, (int)K, gy,
                               s, part);
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
                       (size_t)(4 * hop + GUW) * sizeof(float), st, T, (int)hop, (int)K, F, n, gu, gx, u, gC, ggain);
    return launched("lp_sf_source_adjoint");
}

}  // extern "C"
