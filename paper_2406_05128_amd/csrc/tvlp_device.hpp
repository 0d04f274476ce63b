// Device code of the time-varying LP filter for gfx950 (CDNA4, wave64).
//
// Recursion (paper Sec. 3.2, Eq. 6):  s(t) = e(t) - sum_{i=1..M} a_i(t) s(t-i).
// Adjoint  (Eqs. 12-13):  ghat(t) = g(t) - sum_i a_i(t+i) ghat(t+i),
//                          dL/de(t) = ghat(t),  dL/da_i(t) = -ghat(t) s(t-i).
//
// Chunked linear-recurrence scan.  A sequence is cut into chunks of L samples
// (L a multiple of M, chunk c = [cL, cL+L)).  The state entering chunk c is
// x_c[k] = s(cL-1-k), k = 0..M-1.  By linearity of Eq. 6 the chunk maps it as
//     x_{c+1} = Phi_c x_c + z_c,
// where z_c is the chunk's zero-state response (last M outputs with x_c = 0)
// and column j of Phi_c is its response to the unit state s(cL-1-j) = 1
// (zero input).  Given Phi_c and z_c for every chunk, a short carry over the
// chunks yields all x_c exactly, and each chunk is then rerun from its true
// entry state.  The adjoint runs the transposed ("push") form of Eq. 12 over a
// chunk backwards in time; its pending-contribution vector at the chunk start,
// y_c[j] = dL/ds(cL-1-j) from samples >= cL, obeys y_c = Phi_c^T y_{c+1} + q_c,
// with q_c the chunk's zero-terminal-state adjoint response, so the forward's
// Phi_c serve the reverse carry too.
//
// All arithmetic is float64 (gfx950 issues FP64 FMA at the unpacked FP32
// rate); inputs and outputs are float32.  Register histories are circular
// buffers indexed by time mod M; unrolling time loops by M makes every index a
// compile-time constant so the buffers stay in VGPRs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvlp {

// ---------------------------------------------------------------- sequences

// Either a uniform batch (offsets == nullptr: sequence b = samples [b*T, b*T+T))
// or a packed variable-length batch with device offsets [n+1] and the matching
// chunk prefix cbase [n+1] (cbase[b] = sum of chunk counts of sequences < b).
// For packed batches every sequence view is clamped to [0, N) and every chunk
// index to [0, nch), so malformed offsets cannot address outside the buffers.
struct Seqs {
    const int64_t *offsets;
    const int64_t *cbase;
    // segment-table mode (offsets == nullptr, starts != nullptr): sequence b
    // occupies [starts[b], starts[b] + lens[b]) of the arrays, in any order,
    // possibly with gaps; cbase as for packed batches
    const int64_t *starts;
    const int64_t *lens;
    int64_t T;
    int64_t n;
    int L;
    int64_t N;    // packed samples (varlen only)
    int64_t nch;  // chunk slots allocated (varlen only)
    // uniform batches only: when > 0, sequences b and b + gshare read the same
    // upstream-gradient row (a filter pair sharing dL/dy)
    int64_t gshare;
    // time-invariant coefficients: one row a[b][0..M-1] per sequence, used at
    // every sample of sequence b (uniform batches only)
    int ti;
    // frame-rate coefficients (uniform batches only; hop > 0): rows A[b][q][0..M-1]
    // for q < F, frame q at sample q*hop, linearly interpolated per sample; nf:
    // frame rows one chunk can touch, (L - 1) / hop + 3
    int hop = 0;
    int nf = 0;
    int64_t F = 0;
};

// Coefficient row (in rows of M floats) of the first sample of a chunk of
// sequence b starting at element `start`, and whether rows advance per sample.
__device__ __forceinline__ int64_t coef_row(const Seqs &S, int64_t b, int64_t start) {
    return S.ti ? b : start;
}

// Element offset to add to a sequence's own row index when reading the shared
// upstream-gradient stream (0 unless the batch is a stacked filter pair).
__device__ __forceinline__ int64_t gshare_offset(const Seqs &S, int64_t b) {
    return S.gshare > 0 ? -(b / S.gshare) * S.gshare * S.T : 0;
}

struct SeqView {
    int64_t start;  // element offset of sample 0
    int64_t len;    // samples
    int64_t cbase;  // global index of chunk 0
    int64_t C;      // chunks
};

__device__ __forceinline__ int64_t nchunks_of(int64_t len, int L) {
    return len <= 0 ? 0 : (len + L - 1) / L;
}

__device__ __forceinline__ SeqView seq_view(const Seqs &S, int64_t b) {
    SeqView v;
    if (S.offsets || S.starts) {
        int64_t lo, hi;
        if (S.offsets) {
            lo = min(max(S.offsets[b], (int64_t)0), S.N);
            hi = min(max(S.offsets[b + 1], lo), S.N);
        } else {
            lo = min(max(S.starts[b], (int64_t)0), S.N);
            hi = min(max(lo + S.lens[b], lo), S.N);
        }
        v.start = lo;
        v.len = hi - lo;
        v.cbase = min(max(S.cbase[b], (int64_t)0), S.nch);
        v.C = min(nchunks_of(v.len, S.L), S.nch - v.cbase);
    } else {
        v.start = b * S.T;
        v.len = S.T;
        v.cbase = b * nchunks_of(S.T, S.L);
        v.C = nchunks_of(v.len, S.L);
    }
    return v;
}

// Sequence owning global chunk gc: the largest b with cbase[b] <= gc.
__device__ __forceinline__ int64_t seq_of_chunk(const Seqs &S, int64_t gc) {
    if (!S.cbase) return gc / nchunks_of(S.T, S.L);
    int64_t lo = 0, hi = S.n;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (S.cbase[mid] <= gc) lo = mid; else hi = mid;
    }
    return lo;
}

template <int M>
__device__ __forceinline__ constexpr int wrap(int x) { return ((x % M) + M) % M; }

// Load row t of the coefficient matrix (M float32) and promote to float64.
template <int M>
__device__ __forceinline__ void load_row(const float *__restrict__ row, double (&ad)[M]) {
    if constexpr (M % 2 == 0) {
        const float2 *r2 = reinterpret_cast<const float2 *>(row);
#pragma unroll
        for (int i = 0; i < M / 2; ++i) {
            const float2 v = r2[i];
            ad[2 * i] = (double)v.x;
            ad[2 * i + 1] = (double)v.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < M; ++i) ad[i] = (double)row[i];
    }
}

// y(t) = in - sum_i a_i y(t-i); history h holds y(t-i) at slot (K - i) mod M
// and receives y(t) at slot K.  Two partial sums shorten the FMA chain.
template <int M, int K>
__device__ __forceinline__ double lp_step(double (&h)[M], const double (&ad)[M], double in) {
    double acc0 = in, acc1 = 0.0;
#pragma unroll
    for (int i = 1; i <= M; ++i) {
        if (i & 1) acc0 = fma(-ad[i - 1], h[wrap<M>(K - i)], acc0);
        else       acc1 = fma(-ad[i - 1], h[wrap<M>(K - i)], acc1);
    }
    double y = acc0 + acc1;
    h[K] = y;
    return y;
}

// Runtime-indexed read of a register array without spilling it to scratch.
template <int M>
__device__ __forceinline__ double pick(const double (&h)[M], int idx) {
    double r = 0.0;
#pragma unroll
    for (int p = 0; p < M; ++p) r = (p == idx) ? h[p] : r;
    return r;
}

template <int M, int K0>
struct Unroll {
    template <class F>
    __device__ __forceinline__ static void run(F &&f) {
        if constexpr (K0 < M) {
            f(std::integral_constant<int, K0>{});
            Unroll<M, K0 + 1>::run(f);
        }
    }
};

// ---------------------------------------------------------------- forward

// Rerun one chunk (or a whole sequence) of Eq. 6 from a known entry state.
// x[k] = s(-1-k) relative to the segment start.  Writes s for len samples;
// returns the final state in xf (xf[j] = s(len-1-j)).
template <int M>
__device__ __forceinline__ void run_forward(const float *__restrict__ e, const float *__restrict__ a,
                                            float *__restrict__ s, int64_t len,
                                            const double (&x)[M], double (&xf)[M]) {
    double h[M];
#pragma unroll
    for (int p = 0; p < M; ++p) h[p] = x[M - 1 - p];  // s(-1-k) sits at slot (-1-k) mod M = M-1-k
    for (int64_t t0 = 0; t0 < len; t0 += M) {
        Unroll<M, 0>::run([&](auto kc) {
            constexpr int K = decltype(kc)::value;
            const int64_t t = t0 + K;
            if (t < len) {
                double ad[M];
                load_row<M>(a + t * M, ad);
                double y = lp_step<M, K>(h, ad, (double)e[t]);
                s[t] = (float)y;
            }
        });
    }
    const int r = (int)(len % M);
#pragma unroll
    for (int j = 0; j < M; ++j) xf[j] = pick<M>(h, (r - 1 - j + 2 * M) % M);
}

// Basis pass: lane group of LPC lanes per chunk, CPL columns per lane.
// Column 0 is the zero-state response (input e), column j >= 1 the response
// to the unit state s(cL-j) = 1.  Produces Phi_c[k][j-1] = y_j(L-1-k) and
// z_c[k] = y_0(L-1-k) (k = 0..M-1) for every chunk except a sequence's last.
// ---------------------------------------------------------------- adjoint

// Push form of Eq. 12 over one segment, backwards in time.  Pending
// contributions p(t) live in a circular buffer indexed by u = len-1-t (mod M).
// pin[j] = p(len-1-j) on entry (contributions from after the segment);
// pout[j] = p(-1-j) on exit (what the segment pushes before its start).
// ge (may be null) receives ghat.  With GA, ga receives -ghat(t) s(t-i); the
// segment's s is read from `s` and, for t-i < 0, from the state sx[k] = s(-1-k).
template <int M, bool GA>
__device__ __forceinline__ void run_adjoint(const float *__restrict__ g, const float *__restrict__ a,
                                            int64_t len, const double (&pin)[M], double (&pout)[M],
                                            const float *__restrict__ s, const double (&sx)[M],
                                            float *__restrict__ ge, float *__restrict__ ga) {
    double P[M];
#pragma unroll
    for (int p = 0; p < M; ++p) P[p] = pin[p];  // slot j  <->  u = j  <->  t = len-1-j
    // s history for the coefficient gradient: slot (u+i) mod M holds s(t-i).
    double SH[M];
    if constexpr (GA) {
#pragma unroll
        for (int p = 0; p < M; ++p) {
            const int i = (p == 0) ? M : p;
            const int64_t tt = len - 1 - i;
            SH[p] = tt >= 0 ? (double)s[tt] : sx[-1 - tt];
        }
    }
    for (int64_t u0 = 0; u0 < len; u0 += M) {
        Unroll<M, 0>::run([&](auto kc) {
            constexpr int K = decltype(kc)::value;
            const int64_t u = u0 + K;
            if (u < len) {
                const int64_t t = len - 1 - u;
                double ad[M];
                load_row<M>(a + t * M, ad);
                const double gh = (double)g[t] + P[K];
                P[K] = 0.0;
#pragma unroll
                for (int i = 1; i <= M; ++i) P[wrap<M>(K + i)] = fma(-ad[i - 1], gh, P[wrap<M>(K + i)]);
                if (ge) ge[t] = (float)gh;
                if constexpr (GA) {
#pragma unroll
                    for (int i = 1; i <= M; ++i) ga[t * M + (i - 1)] = (float)(-gh * SH[wrap<M>(K + i)]);
                    // slot (u+1) mod M held s(t-1); next step needs s(t-1-M) there
                    const int64_t tn = t - 1 - M;
                    SH[wrap<M>(K + 1)] = tn >= 0 ? (double)s[tn] : (tn >= -M ? sx[-1 - tn] : 0.0);
                }
            }
        });
    }
    const int r = (int)(len % M);
#pragma unroll
    for (int j = 0; j < M; ++j) pout[j] = pick<M>(P, (r + j) % M);  // p(-1-j) <-> u = len+j
}

// q_c: zero-terminal adjoint response of each chunk, one lane per chunk.
// ---------------------------------------------------------------- sequential baseline

template <int M>
__global__ __launch_bounds__(64) void k_plain_fwd(int64_t B, int64_t T, const float *__restrict__ e,
                                                  const float *__restrict__ a,
                                                  const double *__restrict__ zi,
                                                  float *__restrict__ s, double *__restrict__ zf) {
    const int64_t b = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (b >= B) return;
    double x[M], xf[M];
#pragma unroll
    for (int k = 0; k < M; ++k) x[k] = zi ? zi[b * M + k] : 0.0;
    run_forward<M>(e + b * T, a + b * T * M, s + b * T, T, x, xf);
    if (zf) {
#pragma unroll
        for (int j = 0; j < M; ++j) zf[b * M + j] = xf[j];
    }
}

template <int M, bool GA>
__global__ __launch_bounds__(64) void k_plain_bwd(int64_t B, int64_t T, const float *__restrict__ g,
                                                  const float *__restrict__ a,
                                                  const double *__restrict__ zi,
                                                  const float *__restrict__ s,
                                                  float *__restrict__ ge, float *__restrict__ ga,
                                                  double *__restrict__ gzi) {
    const int64_t b = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (b >= B) return;
    double pin[M], pout[M], sx[M];
#pragma unroll
    for (int j = 0; j < M; ++j) { pin[j] = 0.0; sx[j] = zi ? zi[b * M + j] : 0.0; }
    run_adjoint<M, GA>(g + b * T, a + b * T * M, T, pin, pout, GA ? s + b * T : nullptr, sx,
                       ge ? ge + b * T : nullptr, GA ? ga + b * T * M : nullptr);
    if (gzi) {
#pragma unroll
        for (int j = 0; j < M; ++j) gzi[b * M + j] = pout[j];
    }
}

}  // namespace tvlp
