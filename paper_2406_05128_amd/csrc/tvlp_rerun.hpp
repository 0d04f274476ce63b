// Chunk reruns (G lanes per chunk, DPP butterflies) fed by an LDS row ring.
//
// RowRing streams, for the CPW chunks of a wave, one coefficient row (M floats)
// plus one per-sample scalar (e or g) per step into an LDS ring slot with
// global_load_lds (no VGPRs held for prefetch).  D steps are kept in flight;
// before reading slot u the wave waits until at most DMA_N*(D-1) vector-memory
// operations are outstanding, which is only reached once row u has landed
// (the ring loads are issued unconditionally, one group per step, in order).
//
// Every slot ends with at least one spare DMA lane that reads a zero word from
// device memory, so LDS float ZERO of every slot holds 0: taps beyond M read
// it instead of being masked.
//
// Two kinds of steps share the ring.  While every row a step issues lies
// inside its chunk (the first U steps, U a multiple of NS, below the shortest
// chunk of the wave minus D), each lane's DMA address is advanced by one 64-bit
// add and the ring slot is a compile-time constant of an unrolled block.  The
// remaining steps clamp each lane's row into its chunk (rows outside a chunk are
// never used) and read the slot index at run time.
//
// The compiler models a global_load_lds as a 4-byte LDS store at its pointer,
// not as the 256-byte wave-wide write it is, so it may move the next step's
// DMA above this step's reads of the slot that DMA overwrites.  Every loop over
// ring steps therefore starts each step with a scheduling barrier.
#pragma once

#include <type_traits>

#include "tvlp_systolic.hpp"
#include "tvlp_tiles.hpp"

namespace tvlp {

// s_waitcnt immediate that waits for vmcnt <= n only (gfx9 encoding).
constexpr int waitcnt_vm_only(int n) { return (n & 0xF) | (0x7 << 4) | (0xF << 8) | (((n >> 4) & 0x3) << 14); }

typedef __attribute__((address_space(3))) void lds_void_t;

template <int M, int CPW, bool DESC>
struct RowRing {
    static constexpr int ROWF = CPW * M + CPW;      // floats per step actually used
    static constexpr int DMA_N = ROWF / 64 + 1;     // dword DMA instructions per step (>= 1 spare lane)
    static constexpr int D = (63 / DMA_N) < 15 ? (63 / DMA_N) : 15;
    static constexpr int NS = D + 1;
    static constexpr int SLOT = DMA_N * 64;  // floats per ring slot
    static constexpr int FLOATS = NS * SLOT;
    static constexpr int ZERO = ROWF;  // slot float that always holds 0

    typedef __attribute__((address_space(1))) const char gchar;
    typedef __attribute__((address_space(3))) float lfloat;

    // Per DMA instruction: the lane's row-0 address, its current byte offset,
    // the per-step byte increment and the last valid offset (clamped steps),
    // and the running address (unclamped steps).  Steps walk the rows
    // 0 .. len-1 (descending: len-1 .. 0) and then repeat the last row reached,
    // so every address stays inside the lane's chunk; a lane with no rows, and
    // a spare lane, reads the zero word throughout.
    gchar *base[DMA_N];
    gchar *ptr[DMA_N];
    int off[DMA_N], step[DMA_N], lim[DMA_N];

    // my_base: element index of row 0 of this lane's chunk; my_len: its rows
    // (0 if the lane's chunk is inactive); G: lanes per chunk; zero: a device
    // float holding 0; my_xoff: offset added to my_base for the scalar stream x;
    // my_arow: coefficient row of the chunk's row 0, which advances one row per
    // step unless the coefficients are time-invariant (ti).
    __device__ __forceinline__ void init(const float *a, const float *x, const float *zero, int lane,
                                         int64_t my_base, int64_t my_len, int G, int64_t my_xoff,
                                         int64_t my_arow, bool ti) {
#pragma unroll
        for (int i = 0; i < DMA_N; ++i) {
            const int j = 64 * i + lane;
            int k = 0, f = 0;
            bool coef = false, valid = true;
            if (j < CPW * M) {
                k = j / M;
                f = j % M;
                coef = true;
            } else if (j < ROWF) {
                k = j - CPW * M;
            } else {
                valid = false;
            }
            const int64_t kb = __shfl(my_base, k * G, 64);
            const int64_t kl = __shfl(my_len, k * G, 64);
            const int64_t kx = __shfl(my_xoff, k * G, 64);
            const int64_t ka = __shfl(my_arow, k * G, 64);
            const bool live = valid && kl > 0;
            const float *p0 = !live ? zero : (coef ? a + ka * M + f : x + kb + kx);
            const int st = live ? (coef ? (ti ? 0 : 4 * M) : 4) : 0;
            base[i] = (gchar *)p0;
            step[i] = st;
            lim[i] = live ? st * (int)(kl - 1) : 0;
            off[i] = DESC ? lim[i] : 0;
        }
    }

    // Clamped step: row u into slot u % NS.
    __device__ __forceinline__ void issue(float *ring, int u) {
        lfloat *dst = (lfloat *)ring + (u % NS) * SLOT;
#pragma unroll
        for (int i = 0; i < DMA_N; ++i) {
            __builtin_amdgcn_global_load_lds((const void *)(base[i] + off[i]), (lds_void_t *)(dst + 64 * i), 4, 0,
                                             0);
            off[i] = DESC ? max(off[i] - step[i], 0) : min(off[i] + step[i], lim[i]);
        }
    }
    // Switch to unclamped steps (every row until the switch back lies inside its chunk).
    __device__ __forceinline__ void begin_fast() {
#pragma unroll
        for (int i = 0; i < DMA_N; ++i) ptr[i] = base[i] + off[i];
    }
    // Unclamped step into slot KS.
    template <int KS>
    __device__ __forceinline__ void issue_fast(float *ring) {
        lfloat *dst = (lfloat *)ring + KS * SLOT;
#pragma unroll
        for (int i = 0; i < DMA_N; ++i) {
            __builtin_amdgcn_global_load_lds((const void *)ptr[i], (lds_void_t *)(dst + 64 * i), 4, 0, 0);
            ptr[i] += DESC ? -(int64_t)step[i] : (int64_t)step[i];
        }
    }
    // Back to clamped steps, the next row issued being row n.
    __device__ __forceinline__ void end_fast(int n) {
#pragma unroll
        for (int i = 0; i < DMA_N; ++i) off[i] = DESC ? max(lim[i] - n * step[i], 0) : min(n * step[i], lim[i]);
    }

    __device__ __forceinline__ static void wait() { __builtin_amdgcn_s_waitcnt(waitcnt_vm_only(DMA_N * D)); }
    // After issue(u + D): row u + 1 has landed (rows u+2 .. u+D may still be in flight).
    __device__ __forceinline__ static void wait_next() {
        __builtin_amdgcn_s_waitcnt(waitcnt_vm_only(DMA_N * (D - 1)));
    }
    __device__ __forceinline__ static void drain() { __builtin_amdgcn_s_waitcnt(waitcnt_vm_only(0)); }

    // LDS float indices (within a slot) of the lane's taps r*TPL .. r*TPL+TPL-1
    // (ZERO beyond M) and of its chunk's scalar.
    template <int TPL>
    struct Lanes {
        int tap[TPL];
        int x;
        __device__ __forceinline__ Lanes(int slot, int r) {
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                const int t = r * TPL + m;
                tap[m] = t < M ? slot * M + t : ZERO;
            }
            x = CPW * M + slot;
        }
    };
    // The lane's taps and scalar from ring slot ks (run-time or compile-time), as float64.
    template <int TPL, class KS, class LN>
    __device__ __forceinline__ static void load(const float *ring, KS ks, const LN &ln, double (&av)[TPL],
                                                double &x) {
        static_assert(sizeof(ln.tap) == TPL * sizeof(int), "lane table of another tap count");
        const float *sp = ring + (int)ks * SLOT;
#pragma unroll
        for (int m = 0; m < TPL; ++m) av[m] = (double)sp[ln.tap[m]];
        x = (double)sp[ln.x];
    }
};

// ---------------------------------------------------------------- frame-rate coefficients
//
// Coefficients given once per hop samples (frame q at sample q*hop of its
// sequence) and linearly interpolated per sample,
//   a(q*hop + n) = A[q] + n * (A[q+1] - A[q]) / hop,   0 <= n < hop.
// A wave first stages the frame rows its chunks touch in LDS (per chunk k, nf
// rows starting at the chunk's first frame), then produces one interpolated row
// per ring step with one FMA and one LDS store per 64 words, in place of a DMA
// of the per-sample row.  Every lane word keeps its frame row and slope (float64)
// and its phase offset in registers: at wave-uniform issue count p the phase is
// p + c (descending c - p), an exact integer, and the word is
// fma(phase, slope, row) in float64 rounded once to float32 (the float32
// rounding of the interpolation).  Frame changes happen at a handful of steps
// per chunk, at which the affected words reload from the staged rows.

struct FrameInfo {
    int64_t arow;  // element offset of the chunk's sequence in A (b * F * M)
    int64_t tin;   // in-sequence sample index of the chunk's row 0
    int64_t q0;    // frame of row 0 (staged row 0 of the chunk)
    int64_t len;   // rows of the chunk (0: inactive)
};

// LDS bytes of a wave's staging area: CPW records, then [CPW][nf][M] rows.
__host__ __device__ constexpr size_t frame_lds_bytes(int cpw, int m, int nf) {
    return (size_t)cpw * sizeof(FrameInfo) + (size_t)cpw * nf * m * sizeof(float);
}

__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

// Produces ring words j = 64 i + lane (coefficient f = j % M of chunk j / M)
// for rows issued in order: row u of a chunk is its sample u (ascending) or
// len - 1 - u (descending).  Rows past a chunk's end extrapolate the last
// frame's line (finite values, only ever read by masked steps).
template <int M, int CPW, bool DESC>
struct FrameCoefs {
    static constexpr int NC = (CPW * M + 63) / 64;  // LDS stores per produced row
    static constexpr int NONE = 0x7fffffff;
    typedef __attribute__((address_space(3))) float lfloat;
    double a0[NC], sl[NC];  // frame row, slope per sample
    double ph[NC];          // phase of the next row (an exact integer)
    int ti[NC];  // staged index of the word's current frame row
    int nx[NC];  // issue count at which the word's frame changes (NONE: never)
    int p;       // rows issued so far (wave-uniform)
    int ev;      // smallest nx over the wave
    int hop;
    const float *rows;
    const FrameInfo *info;

    // All 64 lanes call this.  lds: the staging area (frame_lds_bytes); slot /
    // lead: the lane's chunk slot and whether it is the first lane of it;
    // my_b, my_tin, my_len: sequence, first in-sequence sample and rows of the
    // lane's chunk (my_len 0: inactive).
    __device__ __forceinline__ void init(const float *__restrict__ A, const Seqs &S, unsigned char *lds, int lane,
                                         int slot, bool lead, int64_t my_b, int64_t my_tin, int64_t my_len) {
        hop = S.hop;
        const int nfr = S.nf;
        FrameInfo *inf = reinterpret_cast<FrameInfo *>(lds);
        float *st = reinterpret_cast<float *>(lds + CPW * sizeof(FrameInfo));
        if (lead && slot < CPW) {
            FrameInfo fi;
            fi.arow = my_b * S.F * M;
            fi.tin = my_tin;
            fi.q0 = my_tin / hop;
            fi.len = my_len;
            inf[slot] = fi;
        }
        __syncthreads();
        // every load of a round is issued before its LDS writes (one memory
        // latency per round of eight words per lane instead of one per word)
        const int n_all = CPW * nfr * M;
        constexpr int U = 8;
        for (int idx0 = lane; idx0 < n_all; idx0 += 64 * U) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = idx0 + 64 * u;
                v[u] = 0.f;
                if (idx < n_all) {
                    const int k = idx / (nfr * M);
                    const int rem = idx - k * nfr * M;
                    const int qq = rem / M, f = rem - qq * M;
                    const FrameInfo fi = inf[k];
                    if (fi.len > 0) {
                        const int64_t q = min(fi.q0 + qq, S.F - 1);
                        v[u] = A[fi.arow + q * M + f];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = idx0 + 64 * u;
                if (idx < n_all) st[idx] = v[u];
            }
        }
        __syncthreads();
        rows = st;
        info = inf;
        p = 0;
        int mn = NONE;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const int j = 64 * i + lane;
            a0[i] = 0.0;
            sl[i] = 0.0;
            ph[i] = 0.0;
            ti[i] = 0;
            nx[i] = NONE;
            if (j < CPW * M) {
                const int k = j / M, f = j - k * M;
                const FrameInfo fi = inf[k];
                if (fi.len > 0) {
                    const int64_t t0 = fi.tin + (DESC ? fi.len - 1 : 0);
                    const int64_t q = t0 / hop;
                    const int n = (int)(t0 - q * hop);
                    ti[i] = (k * nfr + (int)(q - fi.q0)) * M + f;
                    a0[i] = (double)st[ti[i]];
                    sl[i] = ((double)st[ti[i] + M] - a0[i]) / hop;
                    ph[i] = (double)n;  // phase of row 0
                    // rows until the frame changes: down to phase 0, or up to phase hop - 1
                    const int first = DESC ? n + 1 : hop - n;
                    nx[i] = first < fi.len ? first : NONE;
                }
            }
            mn = min(mn, nx[i]);
        }
        ev = wave_min_i32(mn);
    }

    // The words whose frame changes at row p move to the neighbouring frame.
    __device__ __forceinline__ void advance() {
        const int lane = threadIdx.x & 63;
        int mn = NONE;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            if (nx[i] == p) {
                ti[i] += DESC ? -M : M;
                a0[i] = (double)rows[ti[i]];
                sl[i] = ((double)rows[ti[i] + M] - a0[i]) / hop;
                // phase of row p: ascending 0, descending hop - 1
                ph[i] = DESC ? (double)(hop - 1) : 0.0;
                const int64_t len = info[(64 * i + lane) / M].len;
                nx[i] = (int64_t)p + hop < len ? p + hop : NONE;
            }
            mn = min(mn, nx[i]);
        }
        ev = wave_min_i32(mn);
    }

    // Writes the next row's CPW*M words to dst[0 .. CPW*M) (nothing beyond).
    __device__ __forceinline__ void produce(lfloat *dst) {
        if (p == ev) advance();
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            if (64 * (i + 1) <= CPW * M || 64 * i + lane < CPW * M)
                dst[64 * i + lane] = (float)fma(ph[i], sl[i], a0[i]);
            ph[i] += DESC ? -1.0 : 1.0;
        }
        ++p;
    }
};

// RowRing's interface over frame-rate coefficients: a slot holds the CPW*M
// produced coefficient words ([chunk][M]), the CPW scalars of the step and a
// zero word (ZERO).  The scalars are the only DMA: one instruction per step,
// issued by lanes 0 .. CPW only (lane CPW reads the zero word), so that it
// writes nothing beyond the slot.  DL: steps in flight.
template <int M, int CPW, bool DESC, int DL = 15>
struct FrameRing {
    using FC = FrameCoefs<M, CPW, DESC>;
    static constexpr int NC = FC::NC;
    static constexpr int XOFF = CPW * M;
    static constexpr int D = DL;
    static constexpr int NS = D + 1;
    static constexpr int SLOT = (CPW * M + CPW + 1 + 3) / 4 * 4;
    static constexpr int FLOATS = NS * SLOT;
    static constexpr int ZERO = XOFF + CPW;
    static_assert(CPW < 64, "the scalar DMA needs a spare lane");

    typedef __attribute__((address_space(1))) const char gchar;
    typedef __attribute__((address_space(3))) float lfloat;

    gchar *base;
    gchar *ptr;
    int off, step, lim;
    FC fc;

    // As RowRing::init for the scalar stream x; A: frame rows [B][F][M];
    // my_b / my_tin: the lane's chunk's sequence and first in-sequence sample;
    // lds: the frame staging area.
    __device__ __forceinline__ void init(const float *A, const float *x, const float *zero, int lane, int64_t my_base,
                                         int64_t my_len, int G, int64_t my_xoff, int64_t my_b, int64_t my_tin,
                                         const Seqs &S, unsigned char *lds) {
        const int k = lane < CPW ? lane : 0;
        const int64_t kb = __shfl(my_base, k * G, 64);
        const int64_t kl = __shfl(my_len, k * G, 64);
        const int64_t kx = __shfl(my_xoff, k * G, 64);
        const bool live = lane < CPW && kl > 0;
        base = (gchar *)(live ? x + kb + kx : zero);
        step = live ? 4 : 0;
        lim = live ? 4 * (int)(kl - 1) : 0;
        off = DESC ? lim : 0;
        fc.init(A, S, lds, lane, lane / G, lane % G == 0, my_b, my_tin, my_len);
    }

    __device__ __forceinline__ void issue(float *ring, int u) {
        lfloat *dst = (lfloat *)ring + (u % NS) * SLOT;
        if ((threadIdx.x & 63) <= CPW)
            __builtin_amdgcn_global_load_lds((const void *)(base + off), (lds_void_t *)(dst + XOFF), 4, 0, 0);
        off = DESC ? max(off - step, 0) : min(off + step, lim);
        fc.produce(dst);
    }
    __device__ __forceinline__ void begin_fast() { ptr = base + off; }
    template <int KS>
    __device__ __forceinline__ void issue_fast(float *ring) {
        lfloat *dst = (lfloat *)ring + KS * SLOT;
        if ((threadIdx.x & 63) <= CPW)
            __builtin_amdgcn_global_load_lds((const void *)ptr, (lds_void_t *)(dst + XOFF), 4, 0, 0);
        ptr += DESC ? -(int64_t)step : (int64_t)step;
        fc.produce(dst);
    }
    __device__ __forceinline__ void end_fast(int n) { off = DESC ? max(lim - n * step, 0) : min(n * step, lim); }

    __device__ __forceinline__ static void wait() { __builtin_amdgcn_s_waitcnt(waitcnt_vm_only(D)); }
    __device__ __forceinline__ static void wait_next() { __builtin_amdgcn_s_waitcnt(waitcnt_vm_only(D - 1)); }
    __device__ __forceinline__ static void drain() { __builtin_amdgcn_s_waitcnt(waitcnt_vm_only(0)); }

    template <int TPL>
    struct Lanes {
        int tap[TPL];
        int x;
        __device__ __forceinline__ Lanes(int slot, int r) {
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                const int t = r * TPL + m;
                tap[m] = t < M ? slot * M + t : ZERO;
            }
            x = XOFF + slot;
        }
    };
    template <int TPL, class KS, class LN>
    __device__ __forceinline__ static void load(const float *ring, KS ks, const LN &ln, double (&av)[TPL],
                                                double &x) {
        static_assert(sizeof(ln.tap) == TPL * sizeof(int), "lane table of another tap count");
        const float *sp = ring + (int)ks * SLOT;
#pragma unroll
        for (int m = 0; m < TPL; ++m) av[m] = (double)sp[ln.tap[m]];
        x = (double)sp[ln.x];
    }
};

// Number of leading steps (a multiple of NS) whose issued rows all lie inside
// their chunks: every chunk slot of the wave must be active with at least
// U + D rows.  my_len: the lane's chunk rows (0 if inactive).
template <class RR, int G, int CPW>
__device__ __forceinline__ int fast_steps(int64_t my_len) {
    // a multiple of NS and of G (the unclamped steps end on a G-step boundary)
    constexpr int Q = RR::NS % G == 0 ? RR::NS : (G % RR::NS == 0 ? G : RR::NS * G);
    int mn = 0x7fffffff;
#pragma unroll
    for (int k = 0; k < CPW; ++k) mn = min(mn, __builtin_amdgcn_readlane((int)my_len, k * G));
    const int u = mn - RR::D;
    return u > 0 ? u / Q * Q : 0;
}

// Drives steps u = 0 .. L-1 of a ring loop whose D-row prologue has been
// issued and whose step-0 operands are loaded.  body(u, ks, fast) runs step u;
// ks is the slot of step u + 1 (an integral_constant on unclamped steps) and
// fast is std::true_type on unclamped steps (every chunk of the wave live).
template <class RR, class Body>
__device__ __forceinline__ void ring_loop(RR &rr, float *ring, int L, int U, Body &&body) {
    constexpr int NS = RR::NS, D = RR::D;
    if (U > 0) {
        rr.begin_fast();
        for (int ub = 0; ub < U; ub += NS) {
            Unroll<NS, 0>::run([&](auto kc) {
                constexpr int K = decltype(kc)::value;
                __builtin_amdgcn_sched_barrier(0);  // no DMA above the previous step's LDS reads
                rr.template issue_fast<(K + D) % NS>(ring);
                RR::wait_next();
                body(ub + K, std::integral_constant<int, (K + 1) % NS>{}, std::true_type{});
            });
        }
        rr.end_fast(U + D);
    }
    for (int u = U; u < L; ++u) {
        __builtin_amdgcn_sched_barrier(0);
        rr.issue(ring, u + D);
        RR::wait_next();
        body(u, (u + 1) % NS, std::false_type{});
    }
    RR::drain();
}

// Forward rerun of each chunk from its saved entry state: writes s and, for a
// sequence's last chunk, zf.  Also recomputes s for the adjoint.
// One wave (block `blk`) reruns chunks blk*CPW .. blk*CPW+CPW-1; `ring`: LDS
// of RerunLds<M, G>::BYTES bytes.  xs == nullptr: from the zero state; s ==
// nullptr: no output samples; zall: every chunk's final state, zall[c][k] =
// s(end - 1 - k) (the chunk's zero-state offset z_c when run from zero).
// Row ring of CPW chunks: per-sample rows, or frame-rate rows (FR) interpolated in LDS.
template <int M, int CPW, bool DESC, bool FR>
using RingOf = std::conditional_t<FR, FrameRing<M, CPW, DESC>, RowRing<M, CPW, DESC>>;

// Tile ring of the per-sample-row kernels: NT slots of 8 rows (4 rows for 16
// chunks per wave, to keep the ring near 24 KB at 4 slots).
template <int M, int CPW, bool DESC, int NT = 4>
using TileOf = TileRing<M, CPW, DESC, (CPW >= 16 ? 4 : 8), NT>;

// Tile slots of the adjoint's front launch, whose two kinds of waves share
// every SIMD (about 18 KB of LDS per wave at 3 slots, so that eight fit a CU).
constexpr int FrontTiles = 3;

// Rows of the coefficient array (= samples of the sequence layout).
__device__ __forceinline__ int64_t seq_rows(const Seqs &S) {
    return (S.offsets || S.starts) ? S.N : S.n * S.T;
}

// Shortest chunk of the wave (0 if a slot is inactive); my_len: the lane's chunk rows.
template <int CPW, int G>
__device__ __forceinline__ int wave_min_len(int64_t my_len) {
    int mn = 0x7fffffff;
#pragma unroll
    for (int k = 0; k < CPW; ++k) mn = min(mn, __builtin_amdgcn_readlane((int)my_len, k * G));
    return mn;
}

// LDS bytes of a rerun wave's s staging ([cpw][L] floats), rounded to 16 bytes.
__host__ __device__ constexpr size_t rerun_s_lds_bytes(int cpw, int L) {
    return ((size_t)cpw * (size_t)L * sizeof(float) + 15) & ~(size_t)15;
}

template <int M, int G, bool FR = false, bool TILE = false, int NT = 4>
struct RerunLds {
    static constexpr int BYTES =
        (TILE ? TileOf<M, 64 / G, false, NT>::FLOATS : RingOf<M, 64 / G, false, FR>::FLOATS) * 4;
};

// FR: a holds frame-rate rows [B][F][M] and frl is the frame staging area
// (frame_lds_bytes(64 / G, M, S.nf) bytes of LDS).
// TILE: per-sample rows (not FR, not time-invariant) streamed through the
// tile ring of tvlp_tiles.hpp instead of the row ring.
template <int M, int G, bool FR = false, bool TILE = false, int NT = 4>
__device__ __forceinline__ void rerun_chunks(Seqs S, const float *__restrict__ e, const float *__restrict__ a,
                                             const double *__restrict__ xs, float *__restrict__ s,
                                             double *__restrict__ zf, const float *__restrict__ zero,
                                             int64_t nch, int64_t blk, float *ring,
                                             double *__restrict__ zall = nullptr, unsigned char *frl = nullptr,
                                             float *sst = nullptr, uint32_t *__restrict__ nonfinite = nullptr) {
    constexpr int CPW = 64 / G;
    constexpr int TPL = (M + G - 1) / G;
    static_assert(!(TILE && FR), "frame-rate rows are produced in LDS, not tiled");
    using RR = RingOf<M, CPW, false, FR>;
    using TR = TileOf<M, CPW, false, NT>;
    // unclamped tiles store G consecutive outputs per chunk at a time: a tile
    // must end on such a group's boundary
    static_assert(!TILE || TR::ROWS % G == 0, "tile rows must be a multiple of the lanes per chunk");

    const int lane = threadIdx.x;
    const int slot = lane / G, r = lane % G;
    const int64_t gc = blk * CPW + slot;
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
        hist[m] = (active && k < M && xs) ? xs[gc * M + k] : 0.0;
    }
    const int L = S.L;
    // step u's operands are read from LDS during step u-1
    double av[TPL], ex;
    // With sst ([CPW][L] floats of LDS), s is collected there and written with
    // coalesced stores after the loop (stores inside the ring loop share vmcnt
    // with the row DMA and scatter 8 lanes per chunk over the memory pipeline);
    // without it, s goes straight to memory.
    float *so = s ? (sst ? sst + slot * L : s + base) : nullptr;
    float yk = 0.f;  // unclamped steps: lane r keeps y of the steps u = r (mod G)
    // one step of Eq. 6 on the group's lanes, with the next step's operands
    auto step = [&](int u, const double (&nav)[TPL], double nex, auto fast) {
        double part = 0.0;
#pragma unroll
        for (int m = 0; m < TPL; ++m) part = fma(av[m], hist[m], part);
        const double tot = group_sum<G>(part);  // in every lane of the group
        const double y = ex - tot;
        const double up = dpp_f64<DPP_ROW_SHR1>(hist[TPL - 1]);
        if constexpr (decltype(fast)::value) {
            // one store of G consecutive outputs per chunk every G steps
            const int uk = u & (G - 1);
            yk = (r == uk) ? (float)y : yk;
            if (so && uk == G - 1) so[u - (G - 1) + r] = yk;
#pragma unroll
            for (int m = TPL - 1; m > 0; --m) hist[m] = hist[m - 1];
            hist[0] = (r == 0) ? y : up;
        } else {
            const bool live = u < len;
            if (so && live && r == 0) so[u] = (float)y;
#pragma unroll
            for (int m = TPL - 1; m > 0; --m) hist[m] = live ? hist[m - 1] : hist[m];
            hist[0] = live ? ((r == 0) ? y : up) : hist[0];
        }
#pragma unroll
        for (int m = 0; m < TPL; ++m) av[m] = nav[m];
        ex = nex;
    };
    if constexpr (TILE) {
        TR tr;
        const int delta = tr.init(a, seq_rows(S), e, seq_rows(S), lane, base, len, G, base);
        const typename TR::template Lanes<TPL> ln(slot, r, delta);
        tr.start(ring);
        TR::load(ring, TR::first(), ln, av, ex, r);
        tile_loop(tr, ring, L, wave_min_len<CPW, G>(len), [&](int u, auto ks, auto fast) {
            double nav[TPL], nex;
            TR::load(ring, ks, ln, nav, nex, r);
            step(u, nav, nex, fast);
        });
    } else {
        RR rr;
        if constexpr (FR)
            rr.init(a, e, zero, lane, base, len, G, 0, b, c * S.L, S, frl);
        else
            rr.init(a, e, zero, lane, base, len, G, 0, coef_row(S, b, base), S.ti);
        const typename RR::template Lanes<TPL> ln(slot, r);
        for (int u = 0; u < RR::D; ++u) rr.issue(ring, u);
        RR::wait_next();  // row 0
        RR::load(ring, 0, ln, av, ex);
        ring_loop(rr, ring, L, fast_steps<RR, G, CPW>(len), [&](int u, auto ks, auto fast) {
            double nav[TPL], nex;
            RR::load(ring, ks, ln, nav, nex);
            step(u, nav, nex, fast);
        });
    }
    if (s && sst) {
        // the wave's chunks one after the other, 64 consecutive samples per store;
        // a chunk holding a non-finite output flags its sequence
        __syncthreads();
        for (int k = 0; k < CPW; ++k) {
            const int64_t kb = __shfl(base, k * G, 64);
            const int kl = __shfl((int)len, k * G, 64);
            const int64_t kseq = __shfl(b, k * G, 64);
            bool bad = false;
#pragma unroll 8
            for (int i = lane; i < kl; i += 64) {
                const float v = sst[k * L + i];
                bad |= !__builtin_isfinite(v);
                s[kb + i] = v;
            }
            if (nonfinite && __builtin_amdgcn_ballot_w64(bad) != 0 && lane == 0) atomicOr(nonfinite + kseq, 1u);
        }
    }
    if (zall && active) {
#pragma unroll
        for (int m = 0; m < TPL; ++m) {
            const int k = r * TPL + m;
            if (k < M) zall[gc * M + k] = hist[m];
        }
    }
    if (zf && active) {
        const SeqView v = seq_view(S, b);
        if (c == v.C - 1) {
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                const int k = r * TPL + m;
                if (k < M) zf[b * M + k] = hist[m];
            }
        }
    }
}

template <int M, int G, bool FR = false, bool TILE = false>
__global__ __launch_bounds__(64) void k_fwd_rerun2(Seqs S, const float *__restrict__ e,
                                                   const float *__restrict__ a,
                                                   const double *__restrict__ xs,
                                                   float *__restrict__ s, double *__restrict__ zf,
                                                   const float *__restrict__ zero, int64_t nch,
                                                   uint32_t *__restrict__ nonfinite, int stage_s) {
    __shared__ __attribute__((aligned(16))) float ring[RerunLds<M, G, FR, TILE>::BYTES / 4];
    // dynamic LDS: with stage_s the s staging area [CPW][L] floats (s written with
    // coalesced stores after the loop, else as it is produced), then (FR) the
    // frame staging area
    extern __shared__ __attribute__((aligned(16))) unsigned char rerun_dyn[];
    rerun_chunks<M, G, FR, TILE>(S, e, a, xs, s, zf, zero, nch, blockIdx.x, ring, nullptr,
                                 rerun_dyn + (stage_s ? rerun_s_lds_bytes(64 / G, S.L) : 0),
                                 stage_s ? reinterpret_cast<float *>(rerun_dyn) : nullptr, nonfinite);
}

// Adjoint rerun of each chunk (push form of Eq. 12, descending), from the
// carried pending vector yend[gc] (p(len-1-j) = yend[j]); writes ghat and
// -ghat(t) s(t-i) (Eq. 13).  s of the chunk is read from `s_in` (the stored
// output, or s rerun from the saved entry states by the adjoint's front launch)
// and its M predecessors from the saved entry state xs.  The descending pass
// only leaves ghat in LDS; both gradients are then written by all lanes of the
// wave with coalesced stores.
//
// Dynamic LDS: [CPW][M + L] floats of s (ssh[M + t] = s(t), ssh[M-1-k] =
// s(-1-k)) followed by [CPW][L] floats of ghat (and, with FR, the frame staging
// area at the next 16-byte boundary: emit_frame_lds_offset).
//
// tipart: time-invariant coefficients, each chunk's share of dL/da [nch][M];
// with FR (frame-rate rows in a), each chunk's share of dL/dA for the S.nf
// frames from its first one, [nch][S.nf][M] (ga is then unused).
__host__ __device__ constexpr size_t emit_frame_lds_offset(int cpw, int m, int L) {
    return ((size_t)cpw * (m + 2 * (size_t)L) * sizeof(float) + 15) & ~(size_t)15;
}

template <int M, int G, bool FR = false>
__global__ __launch_bounds__(64) void k_adj_emit2(Seqs S, const float *__restrict__ g,
                                                  const float *__restrict__ a, const float *__restrict__ s_in,
                                                  const double *__restrict__ xs,
                                                  const double *__restrict__ yend,
                                                  float *__restrict__ ge, float *__restrict__ ga,
                                                  double *__restrict__ tipart,
                                                  const float *__restrict__ zero, int64_t nch,
                                                  uint32_t *__restrict__ nonfinite) {
    constexpr int CPW = 64 / G;
    constexpr int TPL = (M + G - 1) / G;
    // frame-rate rows: 12 steps in flight keep four blocks of the training shape per CU
    using RD = std::conditional_t<FR, FrameRing<M, CPW, true, 12>, RowRing<M, CPW, true>>;
    __shared__ __attribute__((aligned(16))) float ring[RD::FLOATS];
    extern __shared__ __attribute__((aligned(16))) float ssh_dyn[];

    const int lane = threadIdx.x;
    const int slot = lane / G, r = lane % G;
    const int L = S.L;
    const int64_t gc = (int64_t)blockIdx.x * CPW + slot;
    bool active = gc < nch;
    int64_t len = 0, base = 0, goff = 0, b = 0, c = 0;
    if (active) {
        b = seq_of_chunk(S, gc);
        const SeqView v = seq_view(S, b);
        c = gc - v.cbase;
        active = c < v.C;
        if (active) {
            base = v.start + c * L;
            len = min((int64_t)L, v.len - c * L);
            goff = gshare_offset(S, b);
        }
    }
    float *ssh = ssh_dyn + slot * (M + L);
    float *gsh_all = ssh_dyn + CPW * (M + L);
    float *gsh = gsh_all + slot * L;
    const typename RD::template Lanes<TPL> ln(slot, r);
    const int U = fast_steps<RD, G, CPW>(len);
    // s of the chunk and its M predecessors into LDS; called once the row ring's
    // first rows are in flight, so both wait on the same memory latencies (the
    // descending pass does not read these rows; the barrier after it publishes them)
    auto load_s = [&]() {
        {
            // the chunk's entry state (M words over G lanes), all loads in flight together
            float xv[(M + G - 1) / G];
#pragma unroll
            for (int q = 0; q < (M + G - 1) / G; ++q) {
                const int k = r + G * q;
                xv[q] = (active && k < M) ? (float)xs[gc * M + k] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < (M + G - 1) / G; ++q) {
                const int k = r + G * q;
                if (k < M) ssh[M - 1 - k] = xv[q];
            }
        }
        {
            // sixteen loads per lane in flight before their LDS writes (one at a time,
            // every load of the chunk's s waited on its own memory latency)
            constexpr int U = 16;
            for (int t0 = r; t0 < L; t0 += U * G) {
                float v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int t = t0 + u * G;
                    v[u] = (active && t < len) ? s_in[base + t] : 0.f;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int t = t0 + u * G;
                    if (t < L) ssh[M + t] = v[u];
                }
            }
        }
    };

    // ---- descending adjoint pass
    double P[TPL], P0 = 0.0;
#pragma unroll
    for (int m = 0; m < TPL; ++m) P[m] = 0.0;
    if (active) {
        P0 = yend[gc * M + 0];
#pragma unroll
        for (int m = 0; m < TPL; ++m) {
            const int i = r * TPL + m + 1;
            P[m] = (i < M) ? yend[gc * M + i] : 0.0;
        }
    }
    RD rd;
    if constexpr (FR)
        rd.init(a, g, zero, lane, base, len, G, goff, b, c * L, S,
                reinterpret_cast<unsigned char *>(ssh_dyn) + emit_frame_lds_offset(CPW, M, L));
    else
        rd.init(a, g, zero, lane, base, len, G, goff, coef_row(S, b, base), S.ti);
    for (int u = 0; u < RD::D; ++u) rd.issue(ring, u);
    load_s();
    RD::wait_next();  // row 0 (sample len - 1)
    double av[TPL], gx;
    RD::load(ring, 0, ln, av, gx);
    float *gw = gsh + (len - 1);  // gw[-u] = ghat(len - 1 - u)
    ring_loop(rd, ring, L, U, [&](int u, auto ks, auto fast) {
        double nav[TPL], ngx;
        RD::load(ring, ks, ln, nav, ngx);
        const double gh = gx + P0;
        double np[TPL];
#pragma unroll
        for (int m = 0; m < TPL; ++m) np[m] = fma(-av[m], gh, P[m]);
        // cross-lane moves by every lane, then the step is committed where valid
        const double down = dpp_f64<DPP_ROW_SHL1>(np[0]);
        const double b0 = group_bcast0<G>(np[0], r);
        if constexpr (decltype(fast)::value) {
            if (r == 0) gw[-u] = (float)gh;
            P0 = b0;
#pragma unroll
            for (int m = 0; m + 1 < TPL; ++m) P[m] = np[m + 1];
            P[TPL - 1] = (r == G - 1) ? 0.0 : down;
        } else {
            const bool live = u < len;
            if (live && r == 0) gw[-u] = (float)gh;
            P0 = live ? b0 : P0;
#pragma unroll
            for (int m = 0; m + 1 < TPL; ++m) P[m] = live ? np[m + 1] : P[m];
            P[TPL - 1] = live ? ((r == G - 1) ? 0.0 : down) : P[TPL - 1];
        }
#pragma unroll
        for (int m = 0; m < TPL; ++m) av[m] = nav[m];
        gx = ngx;
    });
    __syncthreads();

    // ---- frame-rate coefficients: with w = n / hop the chunk's samples t = q*hop + n
    // give dL/dA[q] += sum (1 - w) dL/da(t) and dL/dA[q+1] += sum w dL/da(t), from
    // P = sum -ghat(t) s(t-i) and Q = sum n (-ghat(t) s(t-i)) over each frame's samples
    if constexpr (FR) {
        if (tipart) {
            // The wave walks t over the stretches between consecutive boundaries of
            // any of its chunks (a frame's end or a chunk's end), accumulating
            // without branches; at a boundary only the lanes whose boundary it is
            // flush their shares.  A lane past its chunk's end keeps accumulating
            // (reads stay inside its LDS rows) but never flushes again.
            // Within one frame part (at most hop samples) the products and their
            // sums are float32; the parts are combined in float64.
            constexpr int NONE = 0x7fffffff;
            const int hop = S.hop, nfr = S.nf;
            const int ln = (int)len;  // 0 for an inactive chunk
            float P[TPL], Q[TPL];
            double cr[TPL];
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                P[m] = Q[m] = 0.f;
                cr[m] = 0.0;
            }
            double *out = tipart + gc * nfr * M;
            int n = active ? (int)((c * L) % hop) : 0;  // phase of sample t in its frame
            int qq = 0, t = 0;
            int tb_l = ln > 0 ? min(hop - n, ln) : NONE;  // this lane's next boundary
            int tb = wave_min_i32(tb_l);
            while (tb != NONE) {
                float nd = (float)n;
                const int t_start = t;
#pragma unroll 8
                for (; t < tb; ++t) {
                    const float gt = gsh[t];
                    const float gn = gt * nd;
#pragma unroll
                    for (int m = 0; m < TPL; ++m) {
                        const int i = r * TPL + m;  // tap i + 1
                        const float sv = ssh[M + t - 1 - (i < M ? i : 0)];
                        P[m] = __builtin_fmaf(-gt, sv, P[m]);
                        Q[m] = __builtin_fmaf(-gn, sv, Q[m]);
                    }
                    nd += 1.f;
                }
                n += tb - t_start;
                if (tb_l == tb) {  // the chunk's part of frame q ends here
#pragma unroll
                    for (int m = 0; m < TPL; ++m) {
                        const int i = r * TPL + m;
                        const double qh = (double)Q[m] / hop;
                        if (i < M) out[qq * M + i] = cr[m] + (double)P[m] - qh;
                        cr[m] = qh;
                        P[m] = Q[m] = 0.f;
                    }
                    ++qq;
                    if (n == hop) n = 0;
                    tb_l = t < ln ? min(t + hop - n, ln) : NONE;
                }
                tb = wave_min_i32(tb_l);
            }
            if (active) {
#pragma unroll
                for (int m = 0; m < TPL; ++m) {
                    const int i = r * TPL + m;
                    if (i < M) {
                        out[qq * M + i] = cr[m];
                        for (int z = qq + 1; z < nfr; ++z) out[z * M + i] = 0.0;
                    }
                }
            }
        }
    }

    // ---- time-invariant coefficients: the chunk's share of dL/da_i = -sum_t ghat(t) s(t-i)
    if (!FR && tipart) {
        double acc[TPL];
#pragma unroll
        for (int m = 0; m < TPL; ++m) acc[m] = 0.0;
#pragma unroll 8
        for (int t = 0; t < (int)len; ++t) {
            const double gt = (double)gsh[t];
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                const int i = r * TPL + m;  // tap i + 1
                acc[m] = fma(-gt, (double)ssh[M + t - 1 - (i < M ? i : 0)], acc[m]);
            }
        }
        if (active) {
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                const int i = r * TPL + m;
                if (i < M) tipart[gc * M + i] = acc[m];
            }
        }
    }

    // ---- dL/de(t) = ghat(t), dL/da_i(t) = -ghat(t) s(t-i), chunk by chunk with all lanes;
    // with flags requested, a chunk holding a non-finite gradient value flags its sequence
    auto write_grads = [&](auto checkc) {
        constexpr bool CHECK = decltype(checkc)::value;
        for (int k = 0; k < CPW; ++k) {
            const int kl = (int)__shfl(len, k * G, 64);
            const int64_t kb = __shfl(base, k * G, 64);
            const float *sk = ssh_dyn + k * (M + L);
            const float *gk = gsh_all + k * L;
            bool bad = false;
            if (ge || CHECK)
#pragma unroll 8
                for (int t = lane; t < kl; t += 64) {
                    const float v = gk[t];
                    if constexpr (CHECK) bad |= !__builtin_isfinite(v);
                    if (ge) ge[kb + t] = v;
                }
            if (ga) {
                float *gak = ga + kb * M;
                if (M % 2 == 0 && (reinterpret_cast<uintptr_t>(ga) & 7) == 0) {
                    // pairs of taps (i, i+1) of one row per lane, float2 stores (8-byte aligned: M even);
                    // rounds of four pairs per lane, whose LDS reads are all issued before the
                    // first product (a pair at a time waited for its reads on every store)
                    const int n2 = kl * (M / 2);
                    auto pair = [&](int j, float &gt, float &s0, float &s1) {
                        const int f = 2 * j, t = f / M, i = f - t * M;
                        gt = -gk[t];
                        s0 = sk[M + t - 1 - i];
                        s1 = sk[M + t - 2 - i];
                    };
                    auto put = [&](int j, float gt, float s0, float s1) {
                        float2 v;
                        v.x = gt * s0;
                        v.y = gt * s1;
                        if constexpr (CHECK) bad |= !__builtin_isfinite(v.x) | !__builtin_isfinite(v.y);
                        *reinterpret_cast<float2 *>(gak + 2 * j) = v;
                    };
                    int j = lane;
                    for (; j + 192 < n2; j += 256) {
                        float gt[4], s0[4], s1[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) pair(j + 64 * u, gt[u], s0[u], s1[u]);
#pragma unroll
                        for (int u = 0; u < 4; ++u) put(j + 64 * u, gt[u], s0[u], s1[u]);
                    }
                    for (; j < n2; j += 64) {
                        float gt, s0, s1;
                        pair(j, gt, s0, s1);
                        put(j, gt, s0, s1);
                    }
                } else {
                    const int n = kl * M;
                    for (int f = lane; f < n; f += 64) {
                        const int t = f / M, i = f - t * M;
                        const float v = -gk[t] * sk[M + t - 1 - i];
                        if constexpr (CHECK) bad |= !__builtin_isfinite(v);
                        gak[f] = v;
                    }
                }
            }
            if constexpr (CHECK) {
                const int64_t kseq = __shfl(b, k * G, 64);
                if (__builtin_amdgcn_ballot_w64(bad) != 0 && lane == 0) atomicOr(nonfinite + kseq, 1u);
            }
        }
    };
    if (nonfinite)
        write_grads(std::true_type{});
    else
        write_grads(std::false_type{});
}

// dL/da[b][i] for time-invariant coefficients: the per-chunk shares summed over
// the chunks of sequence b (float64), one block per sequence.
template <int M>
__global__ __launch_bounds__(64) void k_ti_reduce(Seqs S, const double *__restrict__ tipart,
                                                  float *__restrict__ ga) {
    const int64_t b = blockIdx.x;
    const int i = threadIdx.x;
    if (b >= S.n || i >= M) return;
    const SeqView v = seq_view(S, b);
    // eight chunks' loads in flight before they are added, in chunk order
    // (one memory latency per eight chunks instead of one per chunk)
    double sum = 0.0;
    int64_t c = 0;
    for (; c + 8 <= v.C; c += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = tipart[(v.cbase + c + u) * M + i];
#pragma unroll
        for (int u = 0; u < 8; ++u) sum += x[u];
    }
    for (; c < v.C; ++c) sum += tipart[(v.cbase + c) * M + i];
    ga[b * M + i] = (float)sum;
}

// dL/dA[b][q][i] for frame-rate coefficients (uniform batches): the shares of
// the chunks whose staged frames include q, summed in float64.  Chunk c stages
// frames floor(c L / hop) .. + nf - 1.  One thread per output.
template <int M>
__global__ __launch_bounds__(256) void k_frames_reduce(Seqs S, const double *__restrict__ part,
                                                       float *__restrict__ gA) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = S.F * M;
    if (idx >= S.n * per) return;
    const int64_t b = idx / per, rem = idx - b * per;
    const int64_t q = rem / M;
    const int i = (int)(rem - q * M);
    const int64_t L = S.L, hop = S.hop, nfr = S.nf;
    const int64_t C = (S.T + L - 1) / L;
    const int64_t chi = min(C - 1, ((q + 1) * hop - 1) / L);  // last chunk starting at or before frame q
    double sum = 0.0;
    for (int64_t c = chi; c >= 0; --c) {
        const int64_t k = q - (c * L) / hop;
        if (k >= nfr) break;  // earlier chunks stage only earlier frames
        sum += part[((b * C + c) * nfr + k) * M + i];
    }
    gA[idx] = (float)sum;
}

// Time-invariant coefficients: every full chunk of sequence b has the same
// transition, Phi = C^L with C the zero-input step on the state
// x = [s(t-1) .. s(t-M)] (x'[0] = -sum_i a_i x[i-1], x'[k] = x[k-1]).  One
// block per sequence computes it by repeated squaring (float64, in LDS) and
// writes it, column-major, into the slot of every chunk that carries a
// transition.
template <int M>
__global__ __launch_bounds__(256) void k_ti_phi(Seqs S, const float *__restrict__ a, double *__restrict__ phiT) {
    constexpr int MM = M * M;
    __shared__ double R[MM], P[MM], Q[MM];  // column-major: X[j * M + k] = X[k][j]
    const int64_t b = blockIdx.x;
    if (b >= S.n) return;
    const SeqView v = seq_view(S, b);
    const int64_t nt = v.C - 1;  // chunks with a transition
    if (nt <= 0) return;
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int q = tid; q < MM; q += nth) {
        const int j = q / M, k = q % M;
        P[q] = (k == 0) ? -(double)a[b * M + j] : (k == j + 1 ? 1.0 : 0.0);
        R[q] = (k == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    auto mul_into = [&](double *X, const double *Y) {  // X <- X Y
        for (int q = tid; q < MM; q += nth) {
            const int j = q / M, k = q % M;
            // fully unrolled, two partial sums: the LDS reads of the row and
            // column are issued together rather than one dependent pair per tap
            double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                if (i & 1)
                    acc1 = fma(X[i * M + k], Y[j * M + i], acc1);
                else
                    acc0 = fma(X[i * M + k], Y[j * M + i], acc0);
            }
            Q[q] = acc0 + acc1;
        }
        __syncthreads();
        for (int q = tid; q < MM; q += nth) X[q] = Q[q];
        __syncthreads();
    };
    for (int n = S.L; n > 0; n >>= 1) {
        if (n & 1) mul_into(R, P);
        if (n > 1) mul_into(P, P);
    }
    // every transition slot gets the same matrix: each thread keeps its entries
    // in registers and writes them chunk by chunk (coalesced across threads)
    double *dst = phiT + v.cbase * MM;
    for (int q = tid; q < MM; q += nth) {
        const double r = R[q];
        int64_t c = 0;
        for (; c + 4 <= nt; c += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) dst[(c + u) * MM + q] = r;
        }
        for (; c < nt; ++c) dst[c * MM + q] = r;
    }
}

// Zero-state offsets z_c of every chunk (time-invariant forward): the rerun from
// the zero state, keeping only each chunk's final state.
template <int M, int G>
__global__ __launch_bounds__(64) void k_ti_zs(Seqs S, const float *__restrict__ e, const float *__restrict__ a,
                                              double *__restrict__ zbuf, const float *__restrict__ zero,
                                              int64_t nch) {
    __shared__ __attribute__((aligned(16))) float ring[RerunLds<M, G>::BYTES / 4];
    rerun_chunks<M, G>(S, e, a, nullptr, nullptr, nullptr, zero, nch, blockIdx.x, ring, zbuf);
}

}  // namespace tvlp
