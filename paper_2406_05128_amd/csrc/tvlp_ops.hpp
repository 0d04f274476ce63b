// Per-order launch sequences of the chunked filter: the kernels each direction
// launches for one call, with their grids, LDS sizes and workspace regions.
// The host API (tvlp_api.hip) calls them through Ops<M>; tvlp_ops.hip
// instantiates them, one order per translation unit, so that the orders
// compile in parallel.
#pragma once

#include "tvlp.h"
#include "tvlp_carry.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

struct TimingRecord {
    const char *name;
    hipEvent_t start, stop;
};

struct lp_plan {
    int device;
    int M;
    int L;
    int flags;
    // the carry mode was fixed by the caller (a flag at creation or
    // lp_plan_set_carry): the autotuner keeps it
    bool carry_fixed;
    void *ws;
    size_t ws_bytes;
    bool timing;
    // captured graphs that hold this plan's workspace address: while any exist the
    // workspace is neither moved nor freed and the chunk length stays fixed
    int live_graphs;
    std::vector<TimingRecord> pending;
    std::map<std::string, std::pair<double, int64_t>> totals;  // name -> (ms, launches)
};

namespace tvlp_host {

using namespace tvlp;

constexpr int kMaxChunk = 2048;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Brackets kernel launches with hipEvents on their stream when the plan's
// timing switch is on (events are read back by lp_plan_timings).
struct Timer {
    lp_plan *p;
    hipStream_t st;
    TimingRecord cur{};
    void begin(const char *name) {
        if (!p || !p->timing) return;
        cur.name = name;
        if (hipEventCreate(&cur.start) != hipSuccess || hipEventCreate(&cur.stop) != hipSuccess) {
            cur.name = nullptr;
            return;
        }
        (void)hipEventRecord(cur.start, st);
    }
    void end() {
        if (!p || !p->timing || !cur.name) return;
        (void)hipEventRecord(cur.stop, st);
        p->pending.push_back(cur);
        cur.name = nullptr;
    }
};

// Basis-pass mapping of the forward scan for order M: LPC lanes per chunk,
// CPL float64 columns per lane (LPC*CPL >= M+1), R coefficient rows per LDS
// slab (R divides M).
template <int M> struct FwdShape;
#define TVLP_FWD_SHAPE(m, lpc, cpl, r)          \
    template <> struct FwdShape<m> {           \
        static constexpr int LPC = lpc, CPL = cpl, R = r; \
        static constexpr int CPW = 64 / lpc;   \
    };
TVLP_FWD_SHAPE(1, 1, 2, 1)
TVLP_FWD_SHAPE(2, 1, 3, 2)
TVLP_FWD_SHAPE(3, 2, 2, 3)
TVLP_FWD_SHAPE(4, 2, 3, 4)
TVLP_FWD_SHAPE(6, 4, 2, 6)
TVLP_FWD_SHAPE(8, 3, 3, 8)
TVLP_FWD_SHAPE(10, 4, 3, 10)
TVLP_FWD_SHAPE(12, 5, 3, 4)
TVLP_FWD_SHAPE(16, 6, 3, 2)
TVLP_FWD_SHAPE(20, 7, 3, 2)
TVLP_FWD_SHAPE(22, 8, 3, 2)
TVLP_FWD_SHAPE(24, 13, 2, 3)
TVLP_FWD_SHAPE(32, 17, 2, 2)
#undef TVLP_FWD_SHAPE

// Lanes per chunk of the systolic reruns and rows per LDS slab.
template <int M>
struct RerunShape {
    static constexpr int G = M >= 8 ? 8 : 4;
    static constexpr int R = 16;
    static constexpr int CPW = 64 / G;
};

template <int M>
struct Ops {
    using FS = FwdShape<M>;
    // dynamic LDS of the adjoint emit kernel: s and ghat of each of its chunks
    static size_t emit_lds_bytes(int L) { return (size_t)RerunShape<M>::CPW * (M + 2 * (size_t)L) * sizeof(float); }
    // longest chunk whose emit kernel fits the 160 KiB LDS of a CU (with its row ring)
    static int max_chunk() {
        constexpr size_t lds = 160 * 1024;
        constexpr size_t ring = RowRing<M, RerunShape<M>::CPW, false>::FLOATS * sizeof(float);
        const size_t per_l = 2 * RerunShape<M>::CPW * sizeof(float);
        const size_t fixed = ring + (size_t)RerunShape<M>::CPW * M * sizeof(float);
        int L = (int)((lds - fixed) / per_l);
        L = std::min(L, kMaxChunk);
        return L / M * M;
    }
    using RS = RerunShape<M>;

    // Everything one call needs, resolved by the host driver.
    struct Bufs {
        Seqs S;
        Groups gf, gb;
        int64_t nch;
        double *xs, *phiT, *yend, *zbuf, *qbuf;
        double *aggf, *inclf, *aggb, *inclb;  // group maps and group carries
        int *status;
        const float *zero;  // 64 floats of 0 in device memory
        float *sbuf;        // s recomputed by the adjoint (one float per sample slot)
        double *fpart;      // frame-rate coefficients: chunk shares of dL/dA [nch][nf][M]
        int chain;  // chained carry: no matrix products between chunk transitions
        uint32_t *nonfinite;  // [n] per-sequence flags (or null): cleared by the carry, set by the emit
    };

    // Frame-rate coefficients with chunk length L and nf staged frame rows per
    // chunk: whether every kernel's LDS (ring, staging, emit buffers) fits a CU.
    static bool frames_lds_ok(int L, int nf) {
        constexpr size_t lds = 160 * 1024;
        using FSH = FwdScanShape<M, FS::LPC, FS::CPL, FS::R, true>;
        const size_t ff = frame_lds_bytes(FS::CPW, M, nf), fr = frame_lds_bytes(RS::CPW, M, nf);
        const size_t front = std::max<size_t>(BwdScanShape<M, RS::G, RS::R, true>::LDS_BYTES,
                                              RerunLds<M, RS::G, true>::BYTES);
        const size_t rerun = RerunLds<M, RS::G, true>::BYTES + rerun_s_lds_bytes(RS::CPW, L);
        const size_t emit = FrameRing<M, RS::CPW, true, 12>::FLOATS * sizeof(float) +
                            emit_frame_lds_offset(RS::CPW, M, L) + fr;
        return FSH::LDS_BYTES + ff <= lds && front + fr <= lds && rerun + fr <= lds && emit <= lds;
    }

    static void forward(const Bufs &w, const float *e, const float *a, const double *zi, float *s, double *zf,
                        hipStream_t st, Timer &tm);

    // FR: a holds frame-rate rows [B][F][M] (w.S.hop, nf, F set), interpolated in the kernels.
    template <bool FR>
    static void forward_t(const Bufs &w, const float *e, const float *a, const double *zi, float *s, double *zf,
                          hipStream_t st, Timer &tm);

    static void backward(const Bufs &w, const float *g, const float *a, const float *e, const float *s_in,
                         float *ge, float *ga, double *gzi, hipStream_t st, Timer &tm);

    // FR: a holds frame-rate rows and ga receives dL/dA [B][F][M] (chunk shares in
    // w.fpart, then summed per frame).
    template <bool FR>
    static void backward_t(const Bufs &w, const float *g, const float *a, const float *e, const float *s_in,
                           float *ge, float *ga, double *gzi, hipStream_t st, Timer &tm);

    static void plain_fwd(int64_t B, int64_t T, const float *e, const float *a, const double *zi, float *s,
                          double *zf, hipStream_t st);

    static void plain_bwd(int64_t B, int64_t T, const float *g, const float *a, const double *zi, const float *s,
                          float *ge, float *ga, double *gzi, hipStream_t st);
};

}  // namespace tvlp_host
