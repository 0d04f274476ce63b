// Local (wait-free) passes of the chunked scans (gfx950, one wave per group).
//
// Forward (k_fwd_local).  A wave owns a group of CPW consecutive chunks of one
// sequence.  It computes each chunk's transition (Phi_c, z_c) with the basis
// pass (LPC lanes per chunk, CPL float64 columns per lane, coefficient rows
// staged through LDS) and stores Phi_c (column-major) and z_c.
//
// Adjoint (k_bwd_local).  The mirror image: per chunk the zero-terminal
// adjoint response q_c (systolic push form of Eq. 12), stored.
//
// No wave waits on another; group maps (grouped carry), the carries across
// chunks and the per-chunk states are computed afterwards by the carry
// kernels (tvlp_carry.hpp).
#pragma once

#include "tvlp_rerun.hpp"

namespace tvlp {

// Groups of CPW chunks per sequence (uniform batches or varlen prefix gbase).
struct Groups {
    const int64_t *gbase;  // varlen: [n+1] prefix of group counts; nullptr for uniform
    int64_t ngroups;
    int cpw;
};

__device__ __forceinline__ int64_t groups_of(int64_t C, int cpw) { return (C + cpw - 1) / cpw; }

// gid -> (sequence, group index within the sequence), sequence-major.
__device__ __forceinline__ void group_at(const Seqs &S, const Groups &G, int64_t gid, int64_t &b, int64_t &g) {
    if (!G.gbase) {
        const int64_t gp = groups_of(nchunks_of(S.T, S.L), G.cpw);
        b = gid / gp;
        g = gid - b * gp;
        return;
    }
    int64_t lo = 0, hi = S.n;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (G.gbase[mid] <= gid) lo = mid; else hi = mid;
    }
    b = lo;
    g = gid - G.gbase[lo];
}

__device__ __forceinline__ int64_t group_id(const Seqs &S, const Groups &G, int64_t b, int64_t g) {
    if (!G.gbase) return b * groups_of(nchunks_of(S.T, S.L), G.cpw) + g;
    return G.gbase[b] + g;
}

// ---------------------------------------------------------------- small dense helpers in LDS

// y = A x + z for an M x M matrix given column-major (AT[j][i] = A[i][j]); lanes i < M.
template <int M>
__device__ __forceinline__ double matvec_cm(const double *AT, const double *x, double zi_, int i) {
    double acc0 = zi_, acc1 = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const double v = AT[j * M + i] * 1.0;
        if (j & 1) acc1 = fma(v, x[j], acc1);
        else acc0 = fma(v, x[j], acc0);
    }
    return acc0 + acc1;
}

// y = A x + z for A row-major (lanes i < M).
template <int M>
__device__ __forceinline__ double matvec_rm(const double *A, const double *x, double zi_, int i) {
    double acc0 = zi_, acc1 = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if (j & 1) acc1 = fma(A[i * M + j], x[j], acc1);
        else acc0 = fma(A[i * M + j], x[j], acc0);
    }
    return acc0 + acc1;
}

// C = A B for M x M matrices stored column-major (XT[j][i] = X[i][j]).
// Lanes l < M*JP: row i = l % M, columns j = l / M + JP*q.
template <int M>
__device__ __forceinline__ void matmul_cm(const double *AT, const double *BT, double *CT, int lane) {
    constexpr int JP = 64 / M > 0 ? 64 / M : 1;
    if (lane < M * JP) {
        const int i = lane % M, jp = lane / M;
        double arow[M];
#pragma unroll
        for (int m = 0; m < M; ++m) arow[m] = AT[m * M + i];
        for (int j = jp; j < M; j += JP) {
            double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (m & 1) acc1 = fma(arow[m], BT[j * M + m], acc1);
                else acc0 = fma(arow[m], BT[j * M + m], acc0);
            }
            CT[j * M + i] = acc0 + acc1;
        }
    }
}

// C = A B for row-major matrices (lanes l < M*JP: row i, columns j).
template <int M>
__device__ __forceinline__ void matmul_rm(const double *A, const double *B, double *C, int lane) {
    constexpr int JP = 64 / M > 0 ? 64 / M : 1;
    if (lane < M * JP) {
        const int i = lane % M, jp = lane / M;
        double arow[M];
#pragma unroll
        for (int m = 0; m < M; ++m) arow[m] = A[i * M + m];
        for (int j = jp; j < M; j += JP) {
            double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (m & 1) acc1 = fma(arow[m], B[m * M + j], acc1);
                else acc0 = fma(arow[m], B[m * M + j], acc0);
            }
            C[i * M + j] = acc0 + acc1;
        }
    }
}

// ---------------------------------------------------------------- forward scan

template <int M, int LPC, int CPL, int R, bool FR = false>
struct FwdScanShape {
    static constexpr int CPW = 64 / LPC;
    // DMA ring: each step moves one coefficient row (M floats) and one
    // excitation value for each of the CPW chunks into a ring slot of
    // DMA_N x 64 floats; D steps are kept in flight.  FR (frame-rate rows):
    // the ring moves only the excitation (one 64-float slot per step), and an
    // M-step block starting at row t0 first produces the interpolated rows
    // t0+1 .. t0+M (the rows its steps read) into an LDS row buffer of M x CW
    // floats (row t0 was read by the previous block's last step).
    static constexpr int ROWF = CPW * M + CPW;           // floats per step slot actually used
    static constexpr int NC = (CPW * M + 63) / 64;
    static constexpr int CW = (CPW * M + 3) / 4 * 4;     // floats per produced row
    static constexpr int DMA_N = FR ? 1 : (ROWF + 63) / 64;  // dword DMA instructions per step
    static constexpr int D = (63 / DMA_N) < 15 ? (63 / DMA_N) : 15;  // steps in flight (vmcnt <= 63)
    static constexpr int SLOTF = DMA_N * 64;                         // floats per ring slot
    static constexpr int XOFF = FR ? 0 : CPW * M;                    // slot float of chunk 0's excitation
    // ring slots: M when that suffices, so that the slot of row t0 + K in the
    // M-step unrolled loop (t0 a multiple of M) is the constant K
    static constexpr int NS = M >= D + 1 ? M : D + 1;
    static constexpr bool CONST_SLOTS = NS == M;
    static constexpr int RING_BYTES = NS * SLOTF * 4 + (FR ? M * CW * 4 : 0);
    static constexpr int RM = R * M;
    static constexpr bool VEC2 = (M % 2 == 0);
    static constexpr int WORDS = VEC2 ? RM / 2 : RM;
    static constexpr int PER_LANE = (WORDS + LPC - 1) / LPC;
    static constexpr int EPER_LANE = (R + LPC - 1) / LPC;
    static constexpr int STRIDE = ((RM + 1) / 2) * 2 + 2;  // floats per chunk slab
    // chunk slabs, per-row scalars, and a 2-float dummy target for masked writes
    static constexpr int SLAB_BYTES = (CPW * STRIDE + CPW * R + 2) * 4;
    static constexpr int LDS_BYTES = RING_BYTES;
};

// s_waitcnt immediate that waits for vmcnt <= n only (gfx9 encoding).
constexpr int waitcnt_vm(int n) { return (n & 0xF) | (0x7 << 4) | (0xF << 8) | (((n >> 4) & 0x3) << 14); }

// FR: a holds frame-rate rows [B][F][M], interpolated per sample in LDS
// (dynamic LDS: the frame staging area, frame_lds_bytes(CPW, M, S.nf) bytes).
template <int M, int LPC, int CPL, int R, bool FR = false>
__global__ __launch_bounds__(64) void k_fwd_local(
    Seqs S, Groups GR, const float *__restrict__ e, const float *__restrict__ a, double *__restrict__ phiT,
    double *__restrict__ zbuf, const float *__restrict__ zero) {
    using SH = FwdScanShape<M, LPC, CPL, R, FR>;
    constexpr int CPW = SH::CPW;
    static_assert(M % R == 0, "slab rows must divide M");
    __shared__ __attribute__((aligned(16))) unsigned char lds_raw[SH::LDS_BYTES];
    extern __shared__ __attribute__((aligned(16))) unsigned char fwd_dyn[];

    const int lane = threadIdx.x;
    const int64_t gid = blockIdx.x;
    if (gid >= GR.ngroups) return;
    int64_t b, g;
    group_at(S, GR, gid, b, g);
    const SeqView v = seq_view(S, b);
    if (g >= groups_of(v.C, CPW)) return;  // slot beyond the real group count
    const int L = S.L;
    const int64_t c0 = g * CPW;
    const int nbasis = (int)min((int64_t)CPW, v.C - 1 - c0);  // chunks carrying a transition

    // ---- basis pass
    const int slot = lane / LPC, sub = lane % LPC;
    const int64_t c = c0 + slot;
    const bool act = slot < CPW && slot < nbasis;
    double h[CPL][M];
#pragma unroll
    for (int m = 0; m < CPL; ++m) {
        const int col = sub * CPL + m;
#pragma unroll
        for (int p = 0; p < M; ++p) h[m][p] = (col >= 1 && p == M - col) ? 1.0 : 0.0;
    }
    typedef __attribute__((address_space(3))) void lds_void;
    if (nbasis > 0) {
        // Per-lane DMA sources: instruction i, lane l moves ring float j = 64 i + l,
        // which is coefficient (k, f) = (j / M, j % M) for j < CPW*M and the
        // excitation value of chunk j - CPW*M above that.  Rows advance by M floats.
        typedef __attribute__((address_space(1))) const char gchar;
        // per instruction: base address, byte offset of the next row, row step, last valid offset
        gchar *src[SH::DMA_N];
        int off[SH::DMA_N], step[SH::DMA_N], lim[SH::DMA_N];
#pragma unroll
        for (int i = 0; i < SH::DMA_N; ++i) {
            const int j = 64 * i + lane;
            const float *p = zero;  // unused slot words stay zero
            int st = 0;
            if constexpr (FR) {
                if (lane < CPW && lane < nbasis) {  // excitation of chunk `lane`
                    p = e + v.start + (c0 + lane) * L;
                    st = 1;
                }
            } else if (j < CPW * M) {
                const int k = j / M, f = j % M;
                if (k < nbasis) {
                    p = a + coef_row(S, b, v.start + (c0 + k) * L) * M + f;
                    st = S.ti ? 0 : M;
                }
            } else if (j < SH::ROWF) {
                const int k = j - CPW * M;
                if (k < nbasis) {
                    p = e + v.start + (c0 + k) * L;
                    st = 1;
                }
            }
            src[i] = (gchar *)p;
            off[i] = 0;
            step[i] = 4 * st;
            lim[i] = 4 * st * (L - 1);
        }
        float *ring = reinterpret_cast<float *>(lds_raw);
        typedef __attribute__((address_space(3))) float lfloat;
        lfloat *ring_l = (lfloat *)lds_raw;
        constexpr int SLOTF = SH::SLOTF;  // floats per ring slot
        // FR: produced rows t0+1 .. t0+M of the block starting at row t0 (row
        // t0+1+k at k; row 0 alone at 0 before the first block)
        lfloat *rows_l = ring_l + SH::NS * SLOTF;
        const float *rows = ring + SH::NS * SLOTF;
        FrameCoefs<M, CPW, false> fc;
        auto produce_block = [&]() {
#pragma unroll 2
            for (int k = 0; k < M; ++k) fc.produce(rows_l + k * SH::CW);
        };
        if constexpr (FR) {
            fc.init(a, S, fwd_dyn, lane, slot, sub == 0, b, (c0 + slot) * L, act ? L : 0);
            fc.produce(rows_l);
        }
        // Rows are issued in order t = 0, 1, ...; every chunk of the basis pass
        // has exactly L rows, and look-ahead issues past row L-1 repeat that row.
        auto issue = [&](int t, int slotn) {  // row min(t, L-1) of every chunk into ring slot slotn
            lfloat *dst = ring_l + slotn * SLOTF;
#pragma unroll
            for (int i = 0; i < SH::DMA_N; ++i) {
                __builtin_amdgcn_global_load_lds((const void *)(src[i] + off[i]), (lds_void *)(dst + 64 * i), 4,
                                                 0, 0);
                off[i] = min(off[i] + step[i], lim[i]);
            }
        };
        // unclamped issue (the row lies inside the chunk): src itself walks the
        // rows, one 64-bit add per instruction
        auto issue_fast = [&](int slotn) {
            lfloat *dst = ring_l + slotn * SLOTF;
#pragma unroll
            for (int i = 0; i < SH::DMA_N; ++i) {
                __builtin_amdgcn_global_load_lds((const void *)src[i], (lds_void *)(dst + 64 * i), 4, 0, 0);
                src[i] += step[i];
            }
        };
        // row t's coefficients and excitation (ring slot slotn; FR: produced row
        // rk), read during step t-1
        // the excitation word a lane reads: its chunk's for the zero-state column
        // (sub 0), else a slot word that is always zero (ZW), so that the
        // column's start needs no select
        constexpr bool ZW = FR ? (CPW < 64) : (SH::ROWF < SLOTF);
        const int exo = (ZW && sub != 0) ? (FR ? CPW : SH::ROWF) : SH::XOFF + (slot < CPW ? slot : 0);
        auto load_row = [&](int slotn, int rk, float (&rv)[M], float &ex) {
            const float *slotp = ring + slotn * SLOTF;
            const float *row = FR ? rows + rk * SH::CW + (slot < CPW ? slot : 0) * M
                                  : slotp + (slot < CPW ? slot : 0) * M;
#pragma unroll
            for (int i = 0; i < M; ++i) rv[i] = row[i];
            ex = slotp[exo];
        };
        for (int t = 0; t < SH::D; ++t) issue(t, t % SH::NS);
        __builtin_amdgcn_s_waitcnt(waitcnt_vm(SH::DMA_N * (SH::D - 1)));  // row 0 has landed
        float rv[M], ex;
        load_row(0, 0, rv, ex);
        // blocks of M steps whose issued rows (up to t0 + M - 1 + D) all lie inside the chunk
        const int Lfast = SH::CONST_SLOTS && L > SH::D ? (L - SH::D) / M * M : 0;
        int t0 = 0;
        auto block = [&](auto fastc) {
            constexpr bool F = decltype(fastc)::value;
            if constexpr (FR) produce_block();
            Unroll<M, 0>::run([&](auto kc) {
                constexpr int K = decltype(kc)::value;
                const int t = t0 + K;
                __builtin_amdgcn_sched_barrier(0);  // no DMA above the previous step's LDS reads
                // overwrites the slot of row t+D-NS <= t-1, consumed in step t-1
                if constexpr (F)
                    issue_fast((K + SH::D) % SH::NS);
                else
                    issue(t + SH::D, SH::CONST_SLOTS ? (K + SH::D) % SH::NS : (t + SH::D) % SH::NS);
                __builtin_amdgcn_s_waitcnt(waitcnt_vm(SH::DMA_N * (SH::D - 1)));  // row t+1 has landed
                float nrv[M], nex;
                load_row(SH::CONST_SLOTS ? (K + 1) % SH::NS : (t + 1) % SH::NS, K, nrv, nex);
                // one chain per column (CPL independent chains cover the FMA
                // latency), oldest tap first so that the newest output enters last
                double acc[CPL];
#pragma unroll
                for (int m = 0; m < CPL; ++m) acc[m] = m == 0 && (ZW || sub == 0) ? (double)ex : 0.0;
#pragma unroll
                for (int i = M; i >= 1; --i) {
                    const double ai = (double)rv[i - 1];
#pragma unroll
                    for (int m = 0; m < CPL; ++m) acc[m] = fma(-ai, h[m][wrap<M>(K - i)], acc[m]);
                }
#pragma unroll
                for (int m = 0; m < CPL; ++m) h[m][K] = acc[m];
#pragma unroll
                for (int i = 0; i < M; ++i) rv[i] = nrv[i];
                ex = nex;
            });
        };
        if (Lfast > 0) {
            // src moves to the next row to issue (row D: no clamping happened, L > D)
#pragma unroll
            for (int i = 0; i < SH::DMA_N; ++i) {
                src[i] += off[i];
                off[i] = 0;
            }
            for (; t0 < Lfast; t0 += M) block(std::true_type{});
            // src is at row Lfast + D (<= L); offsets relative to it, clamped to row L - 1
#pragma unroll
            for (int i = 0; i < SH::DMA_N; ++i) {
                lim[i] = step[i] * (L - 1 - Lfast - SH::D);
                off[i] = min(0, lim[i]);
            }
        }
        for (; t0 < L; t0 += M) block(std::false_type{});
        __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));  // no look-ahead DMA outlives the wave
        // Phi_c column-major to global (column j-1 = response to unit state s(cL-j)),
        // z_c (zero-state response, column 0) alongside
        if (act) {
#pragma unroll
            for (int m = 0; m < CPL; ++m) {
                const int col = sub * CPL + m;
                if (col >= 1 && col <= M) {
#pragma unroll
                    for (int k = 0; k < M; ++k) phiT[(((v.cbase + c) * M) + (col - 1)) * M + k] = h[m][M - 1 - k];
                } else if (col == 0) {
#pragma unroll
                    for (int k = 0; k < M; ++k) zbuf[(v.cbase + c) * M + k] = h[m][M - 1 - k];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- adjoint scan

// TILE: per-sample rows (not frame-rate, not time-invariant) streamed through
// a descending tile ring of FrontTiles slots (tvlp_tiles.hpp) instead of the
// row ring.
template <int M, int G, int R, bool FR = false, bool TILE = false>
struct BwdScanShape {
    static constexpr int CPW = 64 / G;
    using RD = RingOf<M, CPW, true, FR>;
    using TD = TileOf<M, CPW, true, FrontTiles>;
    static constexpr int RING_BYTES = (TILE ? TD::FLOATS : RD::FLOATS) * 4;
    static constexpr int LDS_BYTES = RING_BYTES;
};

// One wave handles adjoint group tid_; lds_raw: SH::LDS_BYTES bytes of LDS;
// FR: a holds frame-rate rows and frl is the frame staging area.
template <int M, int G, int R, bool FR = false, bool TILE = false>
__device__ __forceinline__ void bwd_local_group(Seqs S, Groups GR, const float *__restrict__ g_in,
                                                const float *__restrict__ a, double *__restrict__ qbuf,
                                                const float *__restrict__ zero, int64_t tid_,
                                                unsigned char *lds_raw, unsigned char *frl = nullptr) {
    static_assert(!(TILE && FR), "frame-rate rows are produced in LDS, not tiled");
    using SH = BwdScanShape<M, G, R, FR, TILE>;
    using RD = typename SH::RD;
    using TD = typename SH::TD;
    constexpr int CPW = SH::CPW;
    constexpr int TPL = (M + G - 1) / G;
    float *ring = reinterpret_cast<float *>(lds_raw);

    const int lane = threadIdx.x;
    if (tid_ >= GR.ngroups) return;
    // reverse order inside each sequence (the last group has the lowest index)
    int64_t b, gr;
    group_at(S, GR, tid_, b, gr);
    const SeqView v = seq_view(S, b);
    const int L = S.L;
    const int64_t ng = groups_of(v.C, CPW);
    if (gr >= ng) return;  // slot beyond the real group count
    const int64_t g = ng - 1 - gr;
    const int64_t c0 = g * CPW;
    const int nk = (int)min((int64_t)CPW, v.C - c0);

    // ---- zero-terminal adjoint per chunk (systolic push form, descending)
    const int slot = lane / G, r = lane % G;
    const int64_t c = c0 + slot;
    const bool act = slot < nk;
    const int64_t base = v.start + c * L;
    const int64_t len = act ? min((int64_t)L, v.len - c * L) : 0;
    double P[TPL], P0 = 0.0;
#pragma unroll
    for (int m = 0; m < TPL; ++m) P[m] = 0.0;
    // one descending step of the chunk's adjoint with row u's taps av and
    // upstream gradient gx
    auto step = [&](int u, const double (&av)[TPL], double gx, auto fast) {
        const double gh = gx + P0;
        double np[TPL];
#pragma unroll
        for (int m = 0; m < TPL; ++m) np[m] = fma(-av[m], gh, P[m]);
        const double down = dpp_f64<DPP_ROW_SHL1>(np[0]);
        const double b0 = group_bcast0<G>(np[0], r);
        if constexpr (decltype(fast)::value) {
            // unclamped steps end before the chunk's first sample
            P0 = b0;
#pragma unroll
            for (int m = 0; m + 1 < TPL; ++m) P[m] = np[m + 1];
            P[TPL - 1] = (r == G - 1) ? 0.0 : down;
        } else {
            // a step inside the chunk shifts the pendings one tap down; the
            // chunk's first sample (u = len - 1) keeps the un-shifted p(-i)
            const bool shift = u + 1 < len, last = u + 1 == len;
            P0 = shift ? b0 : P0;
#pragma unroll
            for (int m = 0; m + 1 < TPL; ++m) P[m] = shift ? np[m + 1] : (last ? np[m] : P[m]);
            P[TPL - 1] = shift ? ((r == G - 1) ? 0.0 : down) : (last ? np[TPL - 1] : P[TPL - 1]);
        }
    };
    if constexpr (TILE) {
        // the shared upstream gradient of a stacked pair has half the rows
        const int64_t grows = S.gshare > 0 ? (int64_t)S.gshare * S.T : seq_rows(S);
        TD td;
        const int delta = td.init(a, seq_rows(S), g_in, grows, lane, base, len, G, base + gshare_offset(S, b));
        const typename TD::template Lanes<TPL> ln(slot, r, delta);
        td.start(ring);
        double av[TPL], gx;
        TD::load(ring, TD::first(), ln, av, gx, r);
        // an unclamped tile must end before every chunk's first sample (u = len - 1,
        // the one step that does not shift)
        tile_loop(td, ring, L, wave_min_len<CPW, G>(len) - 1, [&](int u, auto ks, auto fast) {
            double nav[TPL], ngx;
            TD::load(ring, ks, ln, nav, ngx, r);
            step(u, av, gx, fast);
#pragma unroll
            for (int m = 0; m < TPL; ++m) av[m] = nav[m];
            gx = ngx;
        });
    } else {
        RD rd;
        if constexpr (FR)
            rd.init(a, g_in, zero, lane, base, len, G, gshare_offset(S, b), b, c * L, S, frl);
        else
            rd.init(a, g_in, zero, lane, base, len, G, gshare_offset(S, b), coef_row(S, b, base), S.ti);
        const typename RD::template Lanes<TPL> ln(slot, r);
        for (int u = 0; u < RD::D; ++u) rd.issue(ring, u);
        RD::wait_next();  // row 0 (the chunk's last sample)
        double av[TPL], gx;
        RD::load(ring, 0, ln, av, gx);
        ring_loop(rd, ring, L, fast_steps<RD, G, CPW>(len), [&](int u, auto ks, auto fast) {
            double nav[TPL], ngx;
            RD::load(ring, ks, ln, nav, ngx);
            step(u, av, gx, fast);
#pragma unroll
            for (int m = 0; m < TPL; ++m) av[m] = nav[m];
            gx = ngx;
        });
    }
    // q_c[i-1] = p(-i): lane slot (tap i)
    if (act) {
#pragma unroll
        for (int m = 0; m < TPL; ++m) {
            const int i = r * TPL + m + 1;
            if (i <= M) qbuf[(v.cbase + c) * M + (i - 1)] = P[m];
        }
    }
}

template <int M, int G, int R, bool FR = false, bool TILE = false>
__global__ __launch_bounds__(64) void k_bwd_local(Seqs S, Groups GR, const float *__restrict__ g_in,
                                                  const float *__restrict__ a, double *__restrict__ qbuf,
                                                  const float *__restrict__ zero) {
    __shared__ __attribute__((aligned(16))) unsigned char lds_raw[BwdScanShape<M, G, R, FR, TILE>::LDS_BYTES];
    extern __shared__ __attribute__((aligned(16))) unsigned char bwd_dyn[];  // FR: frame staging
    bwd_local_group<M, G, R, FR, TILE>(S, GR, g_in, a, qbuf, zero, blockIdx.x, lds_raw, bwd_dyn);
}

// The adjoint's local scan together with the recompute of s from the saved
// chunk entry states (into s_out), in one launch: neither needs the other, and
// interleaving their blocks gives every SIMD two independent waves whose
// latencies overlap.  Blocks alternate (scan, rerun) while both kinds remain.
template <int M, int G, int R, bool FR = false, bool TILE = false>
__global__ __launch_bounds__(64) void k_bwd_front(Seqs S, Groups GR, const float *__restrict__ g_in,
                                                  const float *__restrict__ a, double *__restrict__ qbuf,
                                                  const float *__restrict__ zero,
                                                  const float *__restrict__ e, const double *__restrict__ xs,
                                                  float *__restrict__ s_out, int64_t nch) {
    constexpr int B1 = BwdScanShape<M, G, R, FR, TILE>::LDS_BYTES, B2 = RerunLds<M, G, FR, TILE, FrontTiles>::BYTES;
    __shared__ __attribute__((aligned(16))) unsigned char lds_raw[B1 > B2 ? B1 : B2];
    extern __shared__ __attribute__((aligned(16))) unsigned char front_dyn[];  // FR: frame staging
    const int64_t nscan = GR.ngroups, nrun = (nch + 64 / G - 1) / (64 / G);
    const int64_t both = nscan < nrun ? nscan : nrun;
    const int64_t i = blockIdx.x;
    bool scan;
    int64_t j;
    if (i < 2 * both) {
        scan = (i & 1) == 0;
        j = i >> 1;
    } else {
        scan = nscan > nrun;
        j = i - both;
    }
    if (scan)
        bwd_local_group<M, G, R, FR, TILE>(S, GR, g_in, a, qbuf, zero, j, lds_raw, front_dyn);
    else
        rerun_chunks<M, G, FR, TILE, FrontTiles>(S, e, a, xs, s_out, nullptr, zero, nch, j,
                                                 reinterpret_cast<float *>(lds_raw), nullptr, front_dyn);
}

}  // namespace tvlp
