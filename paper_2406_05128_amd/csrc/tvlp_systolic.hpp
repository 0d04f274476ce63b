// Cross-lane helpers for the chunk kernels with G lanes per chunk ("systolic"
// mapping), gfx950 wave64.
//
// A wave handles CPW = 64/G chunks.  Lane r of a chunk's group owns the taps
// i = r*TPL + 1 .. r*TPL + TPL (TPL = ceil(M/G); taps beyond M carry zero
// coefficients).  Forward (Eq. 6): each lane keeps s(t-i) for its own taps;
// the partial sums are added across the group with a DPP butterfly, every lane
// forms s(t), and the history moves one lane up per step.  Adjoint (push form
// of Eq. 12): each lane keeps the pending contributions p(t-i) for its taps;
// ghat(t) = g(t) + p(t), each lane subtracts a_i(t) ghat(t) from its pendings
// (reading the coefficient row t contiguously), and the pendings move one lane
// down per step.  The rows themselves arrive through the LDS row ring of
// tvlp_rerun.hpp.
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

}  // namespace tvlp
