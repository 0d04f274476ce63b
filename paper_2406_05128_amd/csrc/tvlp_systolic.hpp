// Chunk reruns with G lanes per chunk ("systolic" mapping), gfx950 wave64.
//
// A wave handles CPW = 64/G chunks.  Lane r of a chunk's group owns the taps
// i = r*TPL + 1 .. r*TPL + TPL (TPL = ceil(M/G); taps beyond M carry zero
// coefficients).  Forward (Eq. 6): each lane keeps s(t-i) for its own taps;
// the partial sums are added across the group with a DPP butterfly, every lane
// forms s(t), and the history moves one lane up per step.  Adjoint (push form
// of Eq. 12): each lane keeps the pending contributions p(t-i) for its taps;
// ghat(t) = g(t) + p(t), each lane subtracts a_i(t) ghat(t) from its pendings
// (reading the coefficient row t contiguously), and the pendings move one lane
// down per step.  Coefficient rows are staged through LDS in slabs of R rows
// per chunk with register prefetch of the next slab, so global loads are
// coalesced (the G lanes of a group read consecutive words of their chunk).
#pragma once

#include "tvlp_device.hpp"

namespace tvlp {

// ---------------------------------------------------------------- DPP helpers (gfx9 encodings)
constexpr int DPP_QUAD_1032 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_2301 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int DPP_QUAD_0000 = 0x00;        // quad_perm [0,0,0,0]
constexpr int DPP_ROW_SHL1 = 0x101;        // lane i <- lane i+1 within a 16-lane row
constexpr int DPP_ROW_SHR1 = 0x111;        // lane i <- lane i-1 within a 16-lane row
constexpr int DPP_ROW_MIRROR = 0x140;      // lane i <- lane 15-i
constexpr int DPP_ROW_HALF_MIRROR = 0x141; // lane i <- lane 7-i within 8

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, true);
    const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi2, lo2);
}

// Sum over the G lanes of a group; every lane receives the bit-identical total.
template <int G>
__device__ __forceinline__ double group_sum(double x) {
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group size");
    if constexpr (G >= 2) x = x + dpp_f64<DPP_QUAD_1032>(x);
    if constexpr (G >= 4) x = x + dpp_f64<DPP_QUAD_2301>(x);
    if constexpr (G >= 8) x = x + dpp_f64<DPP_ROW_HALF_MIRROR>(x);
    if constexpr (G >= 16) x = x + dpp_f64<DPP_ROW_MIRROR>(x);
    return x;
}

// Value of lane 0 of the group, in every lane of the group.
template <int G>
__device__ __forceinline__ double group_bcast0(double v, int r) {
    if constexpr (G == 1) return v;
    double x = v;
    if constexpr (G >= 2) x = dpp_f64<DPP_QUAD_0000>(v);  // lanes 0-3 <- 0, lanes 4-7 <- 4
    if constexpr (G >= 8) {
        const double y = dpp_f64<DPP_ROW_HALF_MIRROR>(x);  // lanes 4-7 <- lanes 3..0
        x = ((r & 7) < 4) ? x : y;
    }
    if constexpr (G >= 16) {
        const double y = dpp_f64<DPP_ROW_MIRROR>(x);  // lanes 8-15 <- lanes 7..0
        x = (r < 8) ? x : y;
    }
    return x;
}

// ---------------------------------------------------------------- slab staging

// Per-wave LDS staging of R coefficient rows (plus one scalar per row) for each
// of the wave's CPW chunks.  The G lanes of chunk `slot` move that chunk's
// rows only, in 8-byte words when M is even.
template <int M, int G, int R>
struct Slab {
    static constexpr int CPW = 64 / G;
    static constexpr int RM = R * M;
    static constexpr bool VEC2 = (M % 2 == 0);
    static constexpr int WORDS = VEC2 ? RM / 2 : RM;  // load units per chunk
    static constexpr int PER_LANE = (WORDS + G - 1) / G;
    static constexpr int SPER_LANE = (R + G - 1) / G;
    // row stride of chunk slabs in floats: keeps 8-byte alignment and staggers banks
    static constexpr int STRIDE = ((RM + 1) / 2) * 2 + 2;

    float2 pa[PER_LANE];
    float ps[SPER_LANE];

    // Load rows [row0, row0 + R) of the chunk (rows outside [0, len) read as 0).
    __device__ __forceinline__ void prefetch(const float *__restrict__ a, const float *__restrict__ x,
                                             int64_t base, int64_t len, int64_t row0, int r, bool active) {
        const int64_t lo = row0 < 0 ? 0 : row0;
        const int64_t hi = row0 + R < len ? row0 + R : len;
#pragma unroll
        for (int k = 0; k < PER_LANE; ++k) {
            const int w = r + G * k;
            float2 v = make_float2(0.f, 0.f);
            if constexpr (VEC2) {
                const int64_t row = row0 + (2 * w) / M;
                if (active && w < WORDS && row >= lo && row < hi)
                    v = *reinterpret_cast<const float2 *>(a + (base + row0) * M + 2 * w);
            } else {
                const int64_t row = row0 + w / M;
                if (active && w < WORDS && row >= lo && row < hi) v.x = a[(base + row0) * M + w];
            }
            pa[k] = v;
        }
#pragma unroll
        for (int k = 0; k < SPER_LANE; ++k) {
            const int w = r + G * k;
            const int64_t row = row0 + w;
            ps[k] = (active && w < R && row >= lo && row < hi) ? x[base + row] : 0.f;
        }
    }

    __device__ __forceinline__ void commit(float *sa, float *sx, int slot, int r) const {
#pragma unroll
        for (int k = 0; k < PER_LANE; ++k) {
            const int w = r + G * k;
            if (w < WORDS) {
                if constexpr (VEC2) *reinterpret_cast<float2 *>(sa + slot * STRIDE + 2 * w) = pa[k];
                else sa[slot * STRIDE + w] = pa[k].x;
            }
        }
#pragma unroll
        for (int k = 0; k < SPER_LANE; ++k) {
            const int w = r + G * k;
            if (w < R) sx[slot * R + w] = ps[k];
        }
    }
};

// ---------------------------------------------------------------- forward rerun

// Rerun every chunk from its saved entry state and write s (and zf for each
// sequence's last chunk).  Also used to recompute s for the adjoint.
template <int M, int G, int R>
__global__ __launch_bounds__(64) void k_fwd_rerun(Seqs S, const float *__restrict__ e,
                                                  const float *__restrict__ a,
                                                  const double *__restrict__ xs,
                                                  float *__restrict__ s, double *__restrict__ zf,
                                                  int64_t nch) {
    using SL = Slab<M, G, R>;
    constexpr int CPW = SL::CPW;
    constexpr int TPL = (M + G - 1) / G;
    __shared__ __attribute__((aligned(16))) float sa[CPW * SL::STRIDE];
    __shared__ float se[CPW * R];
    __shared__ float so[CPW * R];

    const int lane = threadIdx.x;
    const int slot = lane / G, r = lane % G;
    const int64_t gc = (int64_t)blockIdx.x * CPW + slot;
    bool active = gc < nch;
    int64_t b = 0, c = 0, len = 0, base = 0;
    if (active) {
        b = seq_of_chunk(S, gc);
        const SeqView v = seq_view(S, b);
        c = gc - v.cbase;
        active = c < v.C;
        if (active) {
            base = v.start + c * S.L;
            len = min((int64_t)S.L, v.len - c * S.L);
        }
    }
    double hist[TPL];
#pragma unroll
    for (int m = 0; m < TPL; ++m) {
        const int k = r * TPL + m;
        hist[m] = (active && k < M) ? xs[gc * M + k] : 0.0;
    }
    SL slab;
    slab.prefetch(a, e, base, len, 0, r, active);
    const int L = S.L;
    for (int j0 = 0; j0 < L; j0 += R) {
        slab.commit(sa, se, slot, r);
        __syncthreads();
        if (j0 + R < L) slab.prefetch(a, e, base, len, j0 + R, r, active);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int t = j0 + k;
            double part = 0.0;
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                const int tap = r * TPL + m;
                const float av = (tap < M) ? sa[slot * SL::STRIDE + k * M + tap] : 0.f;
                part = fma((double)av, hist[m], part);
            }
            const double tot = group_sum<G>(part);
            const double y = (double)se[slot * R + k] - tot;
            if (r == 0) so[slot * R + k] = (float)y;
            const double up = dpp_f64<DPP_ROW_SHR1>(hist[TPL - 1]);
            if (t < len) {
#pragma unroll
                for (int m = TPL - 1; m > 0; --m) hist[m] = hist[m - 1];
                hist[0] = (r == 0) ? y : up;
            }
        }
        __syncthreads();
        // coalesced store of the slab's outputs
#pragma unroll
        for (int k = 0; k < SL::SPER_LANE; ++k) {
            const int w = r + G * k;
            if (active && w < R && j0 + w < len) s[base + j0 + w] = so[slot * R + w];
        }
    }
    if (zf && active) {
        const SeqView v = seq_view(S, b);
        if (c == v.C - 1) {
            // lane r slot m holds s(len-1-(r*TPL+m)) = zf[r*TPL+m]
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                const int k = r * TPL + m;
                if (k < M) zf[b * M + k] = hist[m];
            }
        }
    }
}

// ---------------------------------------------------------------- adjoint reruns

// Push form of Eq. 12 over one chunk per group, backwards in time.
// Lane r slot m holds p(t - i), i = r*TPL + m + 1, before step t; every lane
// holds p(t) in P0.  EMIT: the run starts from the carried pending vector
// yend[gc] (p(len-1-j) = yend[j]) and writes ghat and -ghat(t) s(t-i); the
// chunk's s comes from `s` (stored) or is recomputed from xs into LDS.
// Otherwise the run starts from zero and stores q_c[j] = p(-1-j).
template <int M, int G, int R, bool EMIT, bool STORED_S>
__global__ __launch_bounds__(64) void k_adj_rerun(Seqs S, const float *__restrict__ g,
                                                  const float *__restrict__ a,
                                                  const float *__restrict__ e,
                                                  const float *__restrict__ s_in,
                                                  const double *__restrict__ xs,
                                                  const double *__restrict__ yend,
                                                  double *__restrict__ q,
                                                  float *__restrict__ ge, float *__restrict__ ga,
                                                  int64_t nch, int need_first) {
    using SL = Slab<M, G, R>;
    constexpr int CPW = SL::CPW;
    constexpr int TPL = (M + G - 1) / G;
    __shared__ __attribute__((aligned(16))) float sa[CPW * SL::STRIDE];
    __shared__ float sg[CPW * R];
    __shared__ float sge[CPW * R];
    // s for the whole chunk plus M samples of history: ssh[slot][M + t] = s(t)
    constexpr int SSTRIDE = EMIT ? 1 : 0;
    extern __shared__ float ssh_dyn[];
    (void)SSTRIDE;

    const int lane = threadIdx.x;
    const int slot = lane / G, r = lane % G;
    const int L = S.L;
    const int64_t gc = (int64_t)blockIdx.x * CPW + slot;
    bool active = gc < nch;
    int64_t c = 0, len = 0, base = 0;
    if (active) {
        const SeqView v = seq_view(S, seq_of_chunk(S, gc));
        c = gc - v.cbase;
        active = c < v.C && (EMIT || c > 0 || need_first);
        if (active) {
            base = v.start + c * L;
            len = min((int64_t)L, v.len - c * L);
        }
    }
    float *ssh = ssh_dyn + slot * (M + L);

    if constexpr (EMIT) {
        // history part of s: s(-1-k) = xs[k]
        for (int k = r; k < M; k += G) ssh[M - 1 - k] = active ? (float)xs[gc * M + k] : 0.f;
        if constexpr (STORED_S) {
            for (int t = r; t < L; t += G) ssh[M + t] = (active && t < len) ? s_in[base + t] : 0.f;
        } else {
            // recompute s over the chunk from its entry state (systolic forward pass)
            double hist[TPL];
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                const int k = r * TPL + m;
                hist[m] = (active && k < M) ? xs[gc * M + k] : 0.0;
            }
            SL slab;
            slab.prefetch(a, e, base, len, 0, r, active);
            for (int j0 = 0; j0 < L; j0 += R) {
                slab.commit(sa, sg, slot, r);
                __syncthreads();
                if (j0 + R < L) slab.prefetch(a, e, base, len, j0 + R, r, active);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int t = j0 + k;
                    double part = 0.0;
#pragma unroll
                    for (int m = 0; m < TPL; ++m) {
                        const int tap = r * TPL + m;
                        const float av = (tap < M) ? sa[slot * SL::STRIDE + k * M + tap] : 0.f;
                        part = fma((double)av, hist[m], part);
                    }
                    const double tot = group_sum<G>(part);
                    const double y = (double)sg[slot * R + k] - tot;
                    if (r == 0 && t < L) ssh[M + t] = (float)y;
                    const double up = dpp_f64<DPP_ROW_SHR1>(hist[TPL - 1]);
                    if (t < len) {
#pragma unroll
                        for (int m = TPL - 1; m > 0; --m) hist[m] = hist[m - 1];
                        hist[0] = (r == 0) ? y : up;
                    }
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }

    // ---- backward pass (descending t), slabs of R rows counted from the chunk end
    double P[TPL];
    double P0 = 0.0;
#pragma unroll
    for (int m = 0; m < TPL; ++m) P[m] = 0.0;
    if constexpr (EMIT) {
        // p(len-1-j) = yend[j]: P0 = yend[0]; lane slot (tap i) = p(len-1-i) = yend[i]
        if (active) {
            P0 = yend[gc * M + 0];
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                const int i = r * TPL + m + 1;
                P[m] = (i < M) ? yend[gc * M + i] : 0.0;
            }
        }
    }
    SL slab;
    // slab j covers steps u in [j0, j0+R): t = len-1-u, rows [len-j0-R, len-j0)
    slab.prefetch(a, g, base, len, len - R, r, active);
    for (int j0 = 0; j0 < L; j0 += R) {
        slab.commit(sa, sg, slot, r);
        __syncthreads();
        if (j0 + R < L) slab.prefetch(a, g, base, len, len - j0 - 2 * R, r, active);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int u = j0 + k;
            const int64_t t = len - 1 - u;
            const int lr = R - 1 - k;  // slab row of t
            const double gh = (double)sg[slot * R + lr] + P0;
            double np[TPL];
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                const int tap = r * TPL + m;
                float *cell = sa + slot * SL::STRIDE + lr * M + tap;
                const float av = (tap < M) ? *cell : 0.f;
                np[m] = fma(-(double)av, gh, P[m]);
                if constexpr (EMIT) {
                    if (tap < M) {
                        // grad_a(t, i) = -ghat(t) s(t-i) overwrites a(t, i) in the slab
                        const float sv = ssh[M + t - (tap + 1) < 0 ? 0 : M + t - (tap + 1)];
                        *cell = (float)(-gh * (double)sv);
                    }
                }
            }
            if constexpr (EMIT) {
                if (r == 0) sge[slot * R + lr] = (float)gh;
            }
            if (u < len) {
                if (u + 1 < len) {
                    // shift to step t-1: P0 <- p(t-1) = lane 0's np[0]; P[m] <- np[m+1]; last <- lane r+1's np[0]
                    const double down = dpp_f64<DPP_ROW_SHL1>(np[0]);
                    P0 = group_bcast0<G>(np[0], r);
#pragma unroll
                    for (int m = 0; m + 1 < TPL; ++m) P[m] = np[m + 1];
                    P[TPL - 1] = (r == G - 1) ? 0.0 : down;
                } else {
                    // last step of the chunk: keep the un-shifted pendings p(-i)
#pragma unroll
                    for (int m = 0; m < TPL; ++m) P[m] = np[m];
                }
            }
        }
        __syncthreads();
        if constexpr (EMIT) {
            // coalesced write-back of grad_a rows and grad_e for the slab (rows [len-j0-R, len-j0))
            const int64_t row0 = len - j0 - R;
            if (ga) {
#pragma unroll
                for (int k = 0; k < SL::PER_LANE; ++k) {
                    const int w = r + G * k;
                    if (w < SL::WORDS) {
                        if constexpr (SL::VEC2) {
                            const int64_t row = row0 + (2 * w) / M;
                            if (active && row >= 0 && row < len)
                                *reinterpret_cast<float2 *>(ga + (base + row0) * M + 2 * w) =
                                    *reinterpret_cast<const float2 *>(sa + slot * SL::STRIDE + 2 * w);
                        } else {
                            const int64_t row = row0 + w / M;
                            if (active && row >= 0 && row < len)
                                ga[(base + row0) * M + w] = sa[slot * SL::STRIDE + w];
                        }
                    }
                }
            }
            if (ge) {
#pragma unroll
                for (int k = 0; k < SL::SPER_LANE; ++k) {
                    const int w = r + G * k;
                    const int64_t row = row0 + w;
                    if (active && w < R && row >= 0 && row < len) ge[base + row] = sge[slot * R + w];
                }
            }
            __syncthreads();
        }
    }
    if constexpr (!EMIT) {
        // q_c[j] = p(-1-j): lane slot (tap i) holds p(-i) = q[i-1]
        if (active) {
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                const int i = r * TPL + m + 1;
                if (i <= M) q[gc * M + (i - 1)] = P[m];
            }
        }
    }
}

}  // namespace tvlp
