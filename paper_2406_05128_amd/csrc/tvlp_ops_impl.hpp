// Definitions of the per-order launch sequences declared in tvlp_ops.hpp.
#pragma once

#include "tvlp_ops.hpp"

namespace tvlp_host {

// Uniform batches whose sequences fit one chunk (T <= L): no chunk carries a
// transition and the carries reduce to k_single_chunk_states.
inline bool single_chunk(const Seqs &S) { return !S.offsets && !S.starts && S.T <= S.L; }

// Compute units of the current device, cached per device (a launch heuristic
// only: 256 on MI355X, the value assumed when the query fails).
inline int device_cus() {
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cache[dev]) {
        int n = 0;
        cache[dev] = (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
                         ? n
                         : 256;
    }
    return cache[dev];
}

// Rounds in which a grid of one-wave blocks runs when LDS (160 KB per CU on
// gfx950) is what limits the waves per CU.
inline int64_t lds_rounds(int64_t waves, size_t lds_per_wave) {
    const int64_t per_cu = std::max<int64_t>(1, (int64_t)((160 * 1024) / std::max<size_t>(lds_per_wave, 1)));
    const int64_t slots = per_cu * device_cus();
    return (waves + slots - 1) / slots;
}

template <int M>
void Ops<M>::forward(const Bufs &w, const float *e, const float *a, const double *zi, float *s, double *zf,
                    hipStream_t st, Timer &tm) {
    forward_t<false>(w, e, a, zi, s, zf, st, tm);
}

template <int M>
template <bool FR>
void Ops<M>::forward_t(const Bufs &w, const float *e, const float *a, const double *zi, float *s, double *zf,
                  hipStream_t st, Timer &tm) {
    if (w.nch <= 0) return;
    // time-invariant coefficients: one transition per sequence (a matrix power)
    // and the chunks' zero-state offsets; the carry then runs chained
    const bool ti = !FR && w.S.ti;
    const int chain = ti ? 1 : w.chain;
    const size_t dynf = FR ? frame_lds_bytes(FS::CPW, M, w.S.nf) : 0;
    // the forward rerun stages s in LDS (ahead of the FR frame staging) for
    // coalesced stores, unless the staging area would add a round of waves
    const int64_t rwaves = ceil_div(w.nch, RS::CPW);
    const size_t rfix = (FR ? frame_lds_bytes(RS::CPW, M, w.S.nf) : 0) +
                        ((!FR && !ti) ? RerunLds<M, RS::G, false, true>::BYTES : RerunLds<M, RS::G, FR>::BYTES);
    const size_t sstage = rerun_s_lds_bytes(RS::CPW, w.S.L);
    const int stage_s = lds_rounds(rwaves, rfix + sstage) <= lds_rounds(rwaves, rfix) ? 1 : 0;
    const size_t dynr = (FR ? frame_lds_bytes(RS::CPW, M, w.S.nf) : 0) + (stage_s ? sstage : 0);
    if (single_chunk(w.S)) {
        // no transitions: each sequence's only chunk starts from zi (or zero)
        tm.begin("fwd_carry");
        hipLaunchKernelGGL((k_single_chunk_states<M>), dim3((unsigned)ceil_div(w.S.n * M, 256)), dim3(256), 0, st,
                           w.S.n, zi, w.xs, w.nonfinite);
        tm.end();
    } else {
        tm.begin("fwd_scan");
        if (ti) {
            if (w.S.T > w.S.L) {  // some chunk carries a transition (uniform batches)
                hipLaunchKernelGGL((k_ti_zs<M, RS::G>), dim3((unsigned)ceil_div(w.nch, RS::CPW)), dim3(64), 0, st,
                                   w.S, e, a, w.zbuf, w.zero, w.nch);
                hipLaunchKernelGGL((k_ti_phi<M>), dim3((unsigned)w.S.n), dim3(256), 0, st, w.S, a, w.phiT);
            }
        } else {
            hipLaunchKernelGGL((k_fwd_local<M, FS::LPC, FS::CPL, FS::R, FR>), dim3((unsigned)w.gf.ngroups), dim3(64),
                               dynf, st, w.S, w.gf, e, a, w.phiT, w.zbuf, w.zero);
        }
        tm.end();
        tm.begin("fwd_carry");
        const dim3 ct(CarryShape<M>::THREADS);
        if (chain)
            hipLaunchKernelGGL((k_fwd_chain<M>), dim3((unsigned)w.S.n), dim3(CarryShape<M>::CHAIN_THREADS), 0, st,
                               w.S, w.gf, zi, w.phiT, w.zbuf, w.aggf, w.inclf, w.xs, chain, w.nonfinite);
        else {  // group maps, then one block per group: its prefix of group maps, then its chunks
            hipLaunchKernelGGL((k_compose<M, FS::CPW, false>), dim3((unsigned)w.gf.ngroups),
                               dim3(ComposeShape<M>::THREADS), compose_lds_bytes<M>(FS::CPW), st, w.S, w.gf, w.phiT,
                               w.zbuf, w.aggf);
            hipLaunchKernelGGL((k_fwd_carry<M, FS::CPW>), dim3((unsigned)w.gf.ngroups), ct, 0, st, w.S, w.gf, zi,
                               w.phiT, w.zbuf, w.aggf, w.xs, w.nonfinite);
        }
        tm.end();
    }
    tm.begin("fwd_emit");
    if (!FR && !ti)  // per-sample rows: tiled row stream
        hipLaunchKernelGGL((k_fwd_rerun2<M, RS::G, false, true>), dim3((unsigned)ceil_div(w.nch, RS::CPW)),
                           dim3(64), dynr, st, w.S, e, a, w.xs, s, zf, w.zero, w.nch, w.nonfinite, stage_s);
    else
        hipLaunchKernelGGL((k_fwd_rerun2<M, RS::G, FR>), dim3((unsigned)ceil_div(w.nch, RS::CPW)), dim3(64), dynr,
                           st, w.S, e, a, w.xs, s, zf, w.zero, w.nch, w.nonfinite, stage_s);
    tm.end();
}

template <int M>
void Ops<M>::backward(const Bufs &w, const float *g, const float *a, const float *e, const float *s_in,
                     float *ge, float *ga, double *gzi, hipStream_t st, Timer &tm) {
    backward_t<false>(w, g, a, e, s_in, ge, ga, gzi, st, tm);
}

template <int M>
template <bool FR>
void Ops<M>::backward_t(const Bufs &w, const float *g, const float *a, const float *e, const float *s_in,
                   float *ge, float *ga, double *gzi, hipStream_t st, Timer &tm) {
    if (w.nch <= 0) return;
    // without a stored s the emit kernel reads s recomputed alongside the local scan
    const bool emit = ge || ga;
    const float *s_use = s_in ? s_in : w.sbuf;
    const size_t dynr = FR ? frame_lds_bytes(RS::CPW, M, w.S.nf) : 0;
    // per-sample rows (not frame-rate, not time-invariant): tiled row streams
    const bool tile = !FR && !w.S.ti;
    if (emit && s_in && !gzi && single_chunk(w.S)) {
        // one chunk per sequence with s given: the adjoint starts every chunk
        // from the zero terminal state, and no local scan or carry is needed
        tm.begin("bwd_carry");
        hipLaunchKernelGGL((k_single_chunk_states<M>), dim3((unsigned)ceil_div(w.S.n * M, 256)), dim3(256), 0, st,
                           w.S.n, (const double *)nullptr, w.yend, w.nonfinite);
        tm.end();
    } else {
        tm.begin("bwd_scan");
        if (emit && !s_in) {
            const int64_t nrun = ceil_div(w.nch, RS::CPW);
            const dim3 grid((unsigned)(w.gb.ngroups + nrun));
            if (tile)
                hipLaunchKernelGGL((k_bwd_front<M, RS::G, RS::R, FR, !FR>), grid, dim3(64), dynr, st, w.S, w.gb, g, a,
                                   w.qbuf, w.zero, e, w.xs, w.sbuf, w.nch);
            else
                hipLaunchKernelGGL((k_bwd_front<M, RS::G, RS::R, FR>), grid, dim3(64), dynr, st, w.S, w.gb, g, a,
                                   w.qbuf, w.zero, e, w.xs, w.sbuf, w.nch);
        } else if (tile) {
            hipLaunchKernelGGL((k_bwd_local<M, RS::G, RS::R, FR, !FR>), dim3((unsigned)w.gb.ngroups), dim3(64), dynr,
                               st, w.S, w.gb, g, a, w.qbuf, w.zero);
        } else {
            hipLaunchKernelGGL((k_bwd_local<M, RS::G, RS::R, FR>), dim3((unsigned)w.gb.ngroups), dim3(64), dynr, st,
                               w.S, w.gb, g, a, w.qbuf, w.zero);
        }
        tm.end();
        tm.begin("bwd_carry");
        const dim3 ct(CarryShape<M>::THREADS);
        if (!w.chain)  // the groups' reverse maps
            hipLaunchKernelGGL((k_compose<M, RS::CPW, true>), dim3((unsigned)w.gb.ngroups),
                               dim3(ComposeShape<M>::THREADS), compose_lds_bytes<M>(RS::CPW), st, w.S, w.gb, w.phiT,
                               w.qbuf, w.aggb);
        hipLaunchKernelGGL((k_bwd_chain<M>), dim3((unsigned)w.S.n), dim3(CarryShape<M>::CHAIN_THREADS), 0, st, w.S,
                           w.gb, w.phiT, w.qbuf, w.aggb, w.inclb, w.yend, gzi, w.chain, w.nonfinite);
        if (!w.chain)
            hipLaunchKernelGGL((k_bwd_expand<M, RS::CPW>), dim3((unsigned)w.gb.ngroups), ct, 0, st, w.S, w.gb, w.phiT,
                               w.qbuf, w.inclb, w.yend, gzi);
        tm.end();
    }
    if (emit && FR) {
        const unsigned grid = (unsigned)ceil_div(w.nch, RS::CPW);
        const size_t dyn = emit_frame_lds_offset(RS::CPW, M, w.S.L) + dynr;
        tm.begin("bwd_emit");
        hipLaunchKernelGGL((k_adj_emit2<M, RS::G, true>), dim3(grid), dim3(64), dyn, st, w.S, g, a, s_use, w.xs,
                           w.yend, ge, nullptr, ga ? w.fpart : nullptr, w.zero, w.nch, w.nonfinite);
        if (ga) {
            const int64_t nout = w.S.n * w.S.F * M;
            hipLaunchKernelGGL((k_frames_reduce<M>), dim3((unsigned)ceil_div(nout, 256)), dim3(256), 0, st, w.S,
                               w.fpart, ga);
        }
        tm.end();
    } else if (emit) {
        const unsigned grid = (unsigned)ceil_div(w.nch, RS::CPW);
        const size_t dyn = emit_lds_bytes(w.S.L);
        tm.begin("bwd_emit");
        // time-invariant coefficients: per-chunk shares of dL/da (in the q buffer, free
        // once the carry has run) instead of per-sample rows, then a sum per sequence
        const bool ti = w.S.ti && ga;
        hipLaunchKernelGGL((k_adj_emit2<M, RS::G>), dim3(grid), dim3(64), dyn, st, w.S, g, a, s_use,
                           w.xs, w.yend, ge, w.S.ti ? nullptr : ga, ti ? w.qbuf : nullptr, w.zero, w.nch,
                           w.nonfinite);
        if (ti)
            hipLaunchKernelGGL((k_ti_reduce<M>), dim3((unsigned)w.S.n), dim3(64), 0, st, w.S, w.qbuf, ga);
        tm.end();
    }
}

template <int M>
void Ops<M>::plain_fwd(int64_t B, int64_t T, const float *e, const float *a, const double *zi, float *s,
                      double *zf, hipStream_t st) {
    hipLaunchKernelGGL((k_plain_fwd<M>), dim3((unsigned)ceil_div(B, 64)), dim3(64), 0, st, B, T, e, a, zi, s,
                       zf);
}

template <int M>
void Ops<M>::plain_bwd(int64_t B, int64_t T, const float *g, const float *a, const double *zi, const float *s,
                      float *ge, float *ga, double *gzi, hipStream_t st) {
    if (ga)
        hipLaunchKernelGGL((k_plain_bwd<M, true>), dim3((unsigned)ceil_div(B, 64)), dim3(64), 0, st, B, T, g,
                           a, zi, s, ge, ga, gzi);
    else
        hipLaunchKernelGGL((k_plain_bwd<M, false>), dim3((unsigned)ceil_div(B, 64)), dim3(64), 0, st, B, T, g,
                           a, zi, s, ge, ga, gzi);
}

}  // namespace tvlp_host
