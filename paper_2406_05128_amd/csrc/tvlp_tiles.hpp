// Tile ring: per-sample coefficient rows streamed in tiles of R consecutive
// rows per chunk (gfx950 buffer loads straight into LDS).
//
// The row ring of tvlp_rerun.hpp moves one row per chunk per step with dword
// DMA instructions whose 64 lanes scatter over the wave's chunks; at the
// training shape that pattern tops out near 4.5 TB/s.  Here each chunk's R
// rows (R*M*4 contiguous bytes) are fetched as 16-byte pieces by dwordx4
// buffer_load ... lds instructions, one group per tile: whole cache lines per
// chunk, and about 6.5 TB/s for the same chunks.
//
// Layout of one ring slot (floats):
//   [CPW][CF]  coefficient area, CF = R*M + 4: chunk k's pieces, starting at
//              the 16-byte boundary at or below its first row; row i, tap f of
//              the tile sits at k*CF + delta_k + i*M + f (delta_k < 4 is the
//              chunk's misalignment, the same for every tile)
//   [CPW*R]    the per-sample scalar (e or g) of each chunk and row
// The buffer resources are built per wave with their base at or below every
// row the wave needs, and their size ends at the 16-byte block holding the
// array's last byte.  Out-of-range offsets (pieces of rows beyond the array,
// or before the base, as unsigned wrap-around) read zeros without a memory
// access; a 16-byte block that holds a valid byte never leaves that byte's
// page.  Rows outside a chunk are only ever read by masked steps.
//
// Ascending rings cut each chunk into tiles from its first row; descending
// rings from its last row (tile j holds rows len-(j+1)R .. len-jR-1), so that
// step u of every chunk sits at the same place of the same tile.
#pragma once

#include <stdint.h>

#include <type_traits>

#include "tvlp_device.hpp"

namespace tvlp {

// Row KR (0 .. R-1, in processing order) of the tile whose slot starts at
// float tb of the ring.
template <int KR>
struct TileStep {
    int tb;
};

template <int M, int CPW, bool DESC, int R, int NT>
struct TileRing {
    static_assert((R * M) % 4 == 0, "a tile must be a whole number of 16-byte pieces");
    static constexpr int CF = R * M + 4;        // floats per chunk area
    static constexpr int PPC = CF / 4;          // pieces per chunk
    static constexpr int PIECES = CPW * PPC;
    static constexpr int NI = (PIECES + 63) / 64;  // dwordx4 instructions per tile
    static constexpr int SC = CPW * R;             // scalars per tile
    static constexpr int NX = (SC + 63) / 64;      // dword instructions per tile
    static constexpr int NDMA = NI + NX;
    static constexpr int XOFF = CPW * CF;
    static constexpr int SLOT = (XOFF + NX * 64 + 3) / 4 * 4;  // floats per slot
    static constexpr int FLOATS = NT * SLOT;
    static constexpr int ROWS = R, SLOTS = NT;
    static_assert(NDMA * (NT - 1) <= 63, "vmcnt holds at most 63 outstanding instructions");

    typedef __attribute__((address_space(3))) void lds_void;

    __amdgpu_buffer_rsrc_t ra, rx;
    uint32_t voa[NI], vox[NX];

    // All 64 lanes call this.  a: coefficient rows (a_rows rows of M floats); x:
    // the scalar stream (x_len floats); my_row0 / my_x0: row of a and element of
    // x of this lane's chunk's sample 0; my_len: its rows (0: inactive); G:
    // lanes per chunk.  Returns the chunk's misalignment delta (floats) in
    // every lane of its group.
    __device__ __forceinline__ int init(const float *a, int64_t a_rows, const float *x, int64_t x_len, int lane,
                                        int64_t my_row0, int64_t my_len, int G, int64_t my_x0) {
        // wave bases: the lowest first row (scalar) of the active chunks
        int64_t rmin = INT64_MAX, xmin = INT64_MAX;
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
            const int64_t kr = __shfl(my_row0, k * G, 64);
            const int64_t kx = __shfl(my_x0, k * G, 64);
            const int64_t kl = __shfl(my_len, k * G, 64);
            if (kl > 0) {
                rmin = kr < rmin ? kr : rmin;
                xmin = kx < xmin ? kx : xmin;
            }
        }
        if (rmin == INT64_MAX) rmin = xmin = 0;
        const int64_t abase = ((rmin * M * 4) >> 4) << 4;           // bytes, 16-aligned
        const int64_t aend = ((a_rows * M * 4 + 15) >> 4) << 4;      // end of the last 16-byte block
        const int64_t arec = aend - abase;
        ra = __builtin_amdgcn_make_buffer_rsrc((void *)((const char *)a + abase), (short)0,
                                               (int)(arec < 0x7ffffff0 ? arec : 0x7ffffff0), 0x00020000);
        const int64_t xrec = (x_len - xmin) * 4;
        rx = __builtin_amdgcn_make_buffer_rsrc((void *)(x + xmin), (short)0,
                                               (int)(xrec < 0x7ffffff0 ? xrec : 0x7ffffff0), 0x00020000);
        // tile 0 of chunk k starts at row r0 (ascending: its row 0; descending: len - R)
        auto first_row = [&](int64_t row0, int64_t len) { return DESC ? row0 + len - R : row0; };
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int p = 64 * i + lane;
            const int k = p / PPC < CPW ? p / PPC : CPW - 1, q = p % PPC;
            const int64_t kr = __shfl(my_row0, k * G, 64);
            const int64_t kl = __shfl(my_len, k * G, 64);
            int64_t off = 0;
            if (kl > 0) {
                const int64_t b0 = first_row(kr, kl) * M * 4;
                off = ((b0 >> 4) << 4) + 16 * q - abase;
            }
            voa[i] = (uint32_t)off;
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            const int l = 64 * i + lane;
            const int k = l / R < CPW ? l / R : CPW - 1, row = l % R;
            const int64_t kx = __shfl(my_x0, k * G, 64);
            const int64_t kl = __shfl(my_len, k * G, 64);
            vox[i] = kl > 0 ? (uint32_t)((DESC ? kx + kl - R + row : kx + row) - xmin) * 4u : 0u;
        }
        const int64_t b0 = first_row(my_row0, my_len) * M * 4;
        return my_len > 0 ? (int)((b0 - ((b0 >> 4) << 4)) >> 2) : 0;
    }

    // Tile into ring slot sl; offsets move on to the next tile.
    __device__ __forceinline__ void issue(float *ring, int sl) {
        const int lane = threadIdx.x & 63;
        float *dst = ring + sl * SLOT;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            if (64 * (i + 1) <= PIECES || 64 * i + lane < PIECES)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_void *)(dst + 256 * i), 16, voa[i], 0, 0, 0);
            voa[i] += DESC ? (uint32_t)(-(R * M * 4)) : (uint32_t)(R * M * 4);
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            if (64 * (i + 1) <= SC || 64 * i + lane < SC)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (lds_void *)(dst + XOFF + 64 * i), 4, vox[i], 0, 0, 0);
            vox[i] += DESC ? (uint32_t)(-(R * 4)) : (uint32_t)(R * 4);
        }
    }

    // Tiles 0 .. NT-2 in flight and tile 0 landed.
    __device__ __forceinline__ void start(float *ring) {
#pragma unroll
        for (int j = 0; j < NT - 1; ++j) issue(ring, j);
        wait_tile();
    }
    // After a tile issue: all but the newest NT-2 tiles have landed.
    __device__ __forceinline__ static void wait_tile() {
        __builtin_amdgcn_s_waitcnt(waitcnt_vm_tiles(NDMA * (NT - 2)));
    }
    __device__ __forceinline__ static void drain() { __builtin_amdgcn_s_waitcnt(waitcnt_vm_tiles(0)); }
    static constexpr int waitcnt_vm_tiles(int n) {
        return (n & 0xF) | (0x7 << 4) | (0xF << 8) | (((n >> 4) & 0x3) << 14);
    }

    __device__ __forceinline__ static TileStep<0> first() { return TileStep<0>{0}; }

    // LDS float indices of the lane's taps r*TPL .. r*TPL+TPL-1 (taps beyond M
    // read a neighbour and are zeroed by the mask) and of its chunk's scalar,
    // both relative to a tile's row 0.
    template <int TPL>
    struct Lanes {
        int tap[TPL];
        int a1;  // the chunk's tap 1 (a_1), read by every lane of the group
        int x;
        __device__ __forceinline__ Lanes(int slot, int r, int delta) {
            const int k = slot < CPW ? slot : 0;
#pragma unroll
            for (int m = 0; m < TPL; ++m) {
                const int t = r * TPL + m;
                tap[m] = k * CF + delta + (t < M ? t : M - 1);
            }
            a1 = k * CF + delta;
            x = XOFF + k * R;
        }
    };

    // Raw float32 words of row KR: the lane's taps (beyond M: a neighbour, to be
    // masked when converted), the chunk's a_1 and its scalar.
    template <int TPL, int KR, class LN>
    __device__ __forceinline__ static void load_raw(const float *ring, TileStep<KR> st, const LN &ln,
                                                    float (&t)[TPL], float &a1, float &xv) {
        constexpr int ROW = DESC ? R - 1 - KR : KR;
        const float *sp = ring + st.tb;
#pragma unroll
        for (int m = 0; m < TPL; ++m) t[m] = sp[ln.tap[m] + ROW * M];
        a1 = sp[ln.a1 + ROW * M];
        xv = sp[ln.x + ROW];
    }
    // The lane's taps of a raw row as float64, zero beyond M (r: the lane's rank in its group).
    template <int TPL>
    __device__ __forceinline__ static void widen(const float (&t)[TPL], double (&av)[TPL], int r) {
        constexpr int G = 64 / CPW;
#pragma unroll
        for (int m = 0; m < TPL; ++m) {
            if ((G - 1) * TPL + m >= M)
                av[m] = (r * TPL + m < M) ? (double)t[m] : 0.0;
            else
                av[m] = (double)t[m];
        }
    }

    // The lane's taps (float64, zero beyond M) and scalar at row KR of a tile.
    template <int TPL, int KR, class LN>
    __device__ __forceinline__ static void load(const float *ring, TileStep<KR> st, const LN &ln,
                                                double (&av)[TPL], double &xv, int r) {
        constexpr int ROW = DESC ? R - 1 - KR : KR;
        const float *sp = ring + st.tb;
#pragma unroll
        for (int m = 0; m < TPL; ++m) {
            const float v = sp[ln.tap[m] + ROW * M];
            // taps r*TPL + m >= M exist only in the last lanes of a group
            constexpr int G = 64 / CPW;
            if ((G - 1) * TPL + m >= M)
                av[m] = (r * TPL + m < M) ? (double)v : 0.0;
            else
                av[m] = (double)v;
        }
        xv = (double)sp[ln.x + ROW];
    }
};

// Drives steps u = 0 .. ceil(L/R)*R - 1 of a tile ring whose start() has run and
// whose step-0 operands are loaded.  body(u, next, fast) runs step u; next is
// the TileStep of step u + 1 (already landed), fast is std::true_type when every
// chunk of the wave is live for the whole tile (min_len: the wave's shortest
// chunk, 0 if any slot is inactive).  Steps at or beyond a chunk's length must
// be masked by the body on non-fast tiles.
template <class TR, class Body>
__device__ __forceinline__ void tile_loop(TR &tr, float *ring, int L, int min_len, Body &&body) {
    constexpr int RR = TR::ROWS, NT = TR::SLOTS;
    const int ntiles = (L + RR - 1) / RR;
    for (int j = 0; j < ntiles; ++j) {
        __builtin_amdgcn_sched_barrier(0);  // the refill of the oldest slot stays below its last reads
        tr.issue(ring, (j + NT - 1) % NT);
        const int tb = (j % NT) * TR::SLOT, tbn = ((j + 1) % NT) * TR::SLOT;
        auto run = [&](auto fastc) {
            Unroll<RR, 0>::run([&](auto kc) {
                constexpr int K = decltype(kc)::value;
                if constexpr (K == RR - 1) {
                    TR::wait_tile();  // tile j + 1 has landed
                    body(j * RR + K, TileStep<0>{tbn}, fastc);
                } else {
                    body(j * RR + K, TileStep<K + 1>{tb}, fastc);
                }
            });
        };
        if ((j + 1) * RR <= min_len)
            run(std::true_type{});
        else
            run(std::false_type{});
    }
    TR::drain();
}

// As tile_loop, for bodies that read their operands two steps ahead:
// body(u, next2, fast) receives the TileStep of step u + 2, already landed
// (the wait for tile j + 1 moves to its row R - 2).
template <class TR, class Body>
__device__ __forceinline__ void tile_loop2(TR &tr, float *ring, int L, int min_len, Body &&body) {
    constexpr int RR = TR::ROWS, NT = TR::SLOTS;
    static_assert(RR >= 2 && NT >= 3, "two-ahead reads need two rows per tile and three slots");
    const int ntiles = (L + RR - 1) / RR;
    for (int j = 0; j < ntiles; ++j) {
        __builtin_amdgcn_sched_barrier(0);  // the refill of the oldest slot stays below its last reads
        tr.issue(ring, (j + NT - 1) % NT);
        const int tb = (j % NT) * TR::SLOT, tbn = ((j + 1) % NT) * TR::SLOT;
        auto run = [&](auto fastc) {
            Unroll<RR, 0>::run([&](auto kc) {
                constexpr int K = decltype(kc)::value;
                if constexpr (K == RR - 2) TR::wait_tile();  // tile j + 1 has landed
                if constexpr (K + 2 < RR)
                    body(j * RR + K, TileStep<K + 2>{tb}, fastc);
                else
                    body(j * RR + K, TileStep<K + 2 - RR>{tbn}, fastc);
            });
        };
        if ((j + 1) * RR <= min_len)
            run(std::true_type{});
        else
            run(std::false_type{});
    }
    TR::drain();
}

}  // namespace tvlp
