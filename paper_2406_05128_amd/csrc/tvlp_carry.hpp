// Carries across chunks (gfx950).
//
// Forward.  The group maps x(g+1) = P_g x(g) + r_g, applied from x(0) = zi,
// give every group's entry state; the group's chunk transitions x(c+1) =
// Phi_c x(c) + z_c then give every chunk's entry state x_c (the state the
// reruns start from).  k_fwd_carry does both, one block per group.
//
// Adjoint.  The mirror image, right to left: k_bwd_chain (one block per
// sequence) runs the reverse group maps y(g) = Psi_g y(g+1) + w_g from y = 0 at
// the sequence end; k_bwd_expand (one block per group) applies y(c) = Phi_c^T
// y(c+1) + q_c inside each group, writing the pending vector entering every
// chunk from the right, yend[c] = y(c+1), and dL/dzi = y(0).
//
// Chained mode: k_fwd_chain / k_bwd_chain (one block per sequence) apply every
// chunk's transition in turn (no group maps, hence no matrix products) and
// write the per-chunk vectors themselves.
//
// Matrices are staged through LDS in batches by several waves with many loads
// in flight; in the chain kernels three waves stage the next batch while the
// first wave runs the current one.  The carried vector lives in the first
// wave's registers, one entry per lane; every matrix row is one lane's dot
// product.
#pragma once

#include "tvlp_scan.hpp"

namespace tvlp {

// Copies n doubles from global to LDS; thread t of nt cooperating threads.
// Sixteen loads per thread are issued before their LDS writes, so a batch pays
// about one memory latency per sixteen rounds instead of one per element; with
// both addresses 16-byte aligned each load moves two doubles.
__device__ __forceinline__ void stage_doubles(double *dst, const double *__restrict__ src, int64_t n, int t, int nt) {
    constexpr int U = 16;
    if (((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0) {
        const int64_t n2 = n >> 1;
        const double2 *s2 = reinterpret_cast<const double2 *>(src);
        double2 *d2 = reinterpret_cast<double2 *>(dst);
        for (int64_t q0 = t; q0 < n2; q0 += (int64_t)U * nt) {
            double2 r[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = q0 + (int64_t)u * nt;
                r[u] = q < n2 ? s2[q] : double2{0.0, 0.0};
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = q0 + (int64_t)u * nt;
                if (q < n2) d2[q] = r[u];
            }
        }
        if ((n & 1) && t == 0) dst[n - 1] = src[n - 1];
        return;
    }
    for (int64_t q0 = t; q0 < n; q0 += (int64_t)U * nt) {
        double r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = q0 + (int64_t)u * nt;
            r[u] = q < n ? src[q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = q0 + (int64_t)u * nt;
            if (q < n) dst[q] = r[u];
        }
    }
}

// x_j held by lane j, as a wave-uniform value (two scalar lane reads).
__device__ __forceinline__ double lane_value(double x, int j) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, j);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), j);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// One step of a carry, x <- A x + z, for the M-vector x held one entry per
// lane (lane i < M holds x_i and z_i); A[i][j] = A_[i * si + j * sj] in LDS.
// Lane i reads its row of A (independent of x, so the reads are in flight
// while x is broadcast), takes every x_j from lane j by a scalar read, and
// forms its dot product.  Returns the new x_i (lanes >= M: a dummy value).
template <int M>
__device__ __forceinline__ double reg_step(const double *A_, int si, int sj, double x, double z, int lane) {
    const int i = lane < M ? lane : 0;
    double r[M];
#pragma unroll
    for (int j = 0; j < M; ++j) r[j] = A_[i * si + j * sj];
    double acc0 = z, acc1 = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const double xj = lane_value(x, j);
        if (j & 1)
            acc1 = fma(r[j], xj, acc1);
        else
            acc0 = fma(r[j], xj, acc0);
    }
    return acc0 + acc1;
}

template <int M>
struct CarryShape {
    static constexpr int MM = M * M;
    static constexpr int THREADS = 256;         // expand kernels: four waves
    static constexpr int CHAIN_THREADS = 512;   // chain kernels: one wave computes, seven stage
    static constexpr int BUF_DOUBLES = 8000;    // one chain-kernel staging buffer (62.5 KiB)
    // matrices (each with its offset vector) per chain-kernel batch
    static constexpr int NB = BUF_DOUBLES / (MM + M) > 0 ? BUF_DOUBLES / (MM + M) : 1;
};

// ---------------------------------------------------------------- forward

// Chained: items are chunks (matrix Phi_c, offset z_c; output xs per chunk);
// grouped: items are groups (map with its offset; output ginc per group).
// The last item has no map.
template <int M>
__global__ __launch_bounds__(512) void k_fwd_chain(Seqs S, Groups GR, const double *__restrict__ zi,
                                                   const double *__restrict__ phiT,
                                                   const double *__restrict__ zbuf,
                                                   const double *__restrict__ aggbuf, double *__restrict__ ginc,
                                                   double *__restrict__ xs, int chain,
                                                   uint32_t *__restrict__ nonfinite) {
    using CS = CarryShape<M>;
    constexpr int MM = M * M;
    __shared__ __attribute__((aligned(16))) double lds[2 * CS::BUF_DOUBLES];
    const int64_t b = blockIdx.x;
    if (nonfinite && threadIdx.x == 0) nonfinite[b] = 0u;  // the forward emit sets it
    const SeqView sv = seq_view(S, b);
    if (sv.C <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t n = chain ? sv.C : groups_of(sv.C, GR.cpw);
    const int64_t id0 = chain ? sv.cbase : group_id(S, GR, b, 0);
    double *out = chain ? xs : ginc;
    const int64_t nbatch = (n + CS::NB - 1) / CS::NB;
    auto stage = [&](int64_t bi, int t, int nt) {
        double *buf = lds + (bi & 1) * CS::BUF_DOUBLES;
        const int64_t k0 = bi * CS::NB;
        const int64_t nm = min((int64_t)CS::NB, n - 1 - k0);  // items with a map
        if (chain) {
            stage_doubles(buf, phiT + (id0 + k0) * MM, nm * MM, t, nt);
            stage_doubles(buf + CS::NB * MM, zbuf + (id0 + k0) * M, nm * M, t, nt);
        } else {
            stage_doubles(buf, aggbuf + (id0 + k0) * (MM + M), nm * (MM + M), t, nt);
        }
    };
    double x = (wv == 0 && lane < M && zi) ? zi[b * M + lane] : 0.0;
    stage(0, tid, CS::CHAIN_THREADS);
    __syncthreads();
    for (int64_t bi = 0; bi < nbatch; ++bi) {
        if (wv == 0) {
            const double *buf = lds + (bi & 1) * CS::BUF_DOUBLES;
            const int64_t k0 = bi * CS::NB;
            const int nb = (int)min((int64_t)CS::NB, n - k0);
            for (int k = 0; k < nb; ++k) {
                if (lane < M) out[(id0 + k0 + k) * M + lane] = x;
                if (k0 + k + 1 < n) {
                    const double *A = chain ? buf + k * MM : buf + k * (MM + M);
                    const double *z = chain ? buf + CS::NB * MM + k * M : A + MM;
                    x = reg_step<M>(A, 1, M, x, z[lane < M ? lane : 0], lane);
                }
            }
        } else if (bi + 1 < nbatch) {
            stage(bi + 1, tid - 64, CS::CHAIN_THREADS - 64);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- adjoint

// Chained: items are chunks (Phi_c^T, q_c; output yend per chunk; the last
// chunk has no transition, y = q there); grouped: items are groups (reverse
// map with its offset; output ginc per group; group 0 has no map).  Items are
// visited from the last one down.
template <int M>
__global__ __launch_bounds__(512) void k_bwd_chain(Seqs S, Groups GR, const double *__restrict__ phiT,
                                                   const double *__restrict__ qbuf,
                                                   const double *__restrict__ aggbuf, double *__restrict__ ginc,
                                                   double *__restrict__ yend, double *__restrict__ grad_zi,
                                                   int chain, uint32_t *__restrict__ nonfinite) {
    using CS = CarryShape<M>;
    constexpr int MM = M * M;
    __shared__ __attribute__((aligned(16))) double lds[2 * CS::BUF_DOUBLES];
    const int64_t b = blockIdx.x;
    if (nonfinite && threadIdx.x == 0) nonfinite[b] = 0u;  // the adjoint emit sets it
    const SeqView sv = seq_view(S, b);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (sv.C <= 0) {  // no samples: no dependence on the initial state
        if (grad_zi && tid < M) grad_zi[b * M + tid] = 0.0;
        return;
    }
    const int64_t n = chain ? sv.C : groups_of(sv.C, GR.cpw);
    const int64_t id0 = chain ? sv.cbase : group_id(S, GR, b, 0);
    double *out = chain ? yend : ginc;
    const int64_t nbatch = (n + CS::NB - 1) / CS::NB;
    // batch bi holds items [k0, k0 + nb) with k0 + nb = n - bi * NB
    auto range = [&](int64_t bi, int64_t &k0, int &nb) {
        const int64_t k1 = n - bi * CS::NB;
        nb = (int)min((int64_t)CS::NB, k1);
        k0 = k1 - nb;
    };
    auto stage = [&](int64_t bi, int t, int nt) {
        double *buf = lds + (bi & 1) * CS::BUF_DOUBLES;
        int64_t k0;
        int nb;
        range(bi, k0, nb);
        if (chain) {
            stage_doubles(buf, phiT + (id0 + k0) * MM, (int64_t)nb * MM, t, nt);
            stage_doubles(buf + CS::NB * MM, qbuf + (id0 + k0) * M, (int64_t)nb * M, t, nt);
        } else {
            stage_doubles(buf, aggbuf + (id0 + k0) * (MM + M), (int64_t)nb * (MM + M), t, nt);
        }
    };
    double x = 0.0;
    stage(0, tid, CS::CHAIN_THREADS);
    __syncthreads();
    for (int64_t bi = 0; bi < nbatch; ++bi) {
        if (wv == 0) {
            const double *buf = lds + (bi & 1) * CS::BUF_DOUBLES;
            int64_t k0;
            int nb;
            range(bi, k0, nb);
            for (int k = nb - 1; k >= 0; --k) {
                const int64_t item = k0 + k;
                if (lane < M) out[(id0 + item) * M + lane] = x;
                if (chain) {
                    const double q = buf[CS::NB * MM + k * M + (lane < M ? lane : 0)];
                    if (item == n - 1)
                        x = q;
                    else
                        x = reg_step<M>(buf + k * MM, M, 1, x, q, lane);
                } else if (item > 0) {
                    const double *A = buf + k * (MM + M);
                    x = reg_step<M>(A, M, 1, x, A[MM + (lane < M ? lane : 0)], lane);
                }
            }
            if (chain && bi + 1 == nbatch && grad_zi && lane < M) grad_zi[b * M + lane] = x;
        } else if (bi + 1 < nbatch) {
            stage(bi + 1, tid - 64, CS::CHAIN_THREADS - 64);
        }
        __syncthreads();
    }
}

template <int M, int CPW>
__global__ __launch_bounds__(256) void k_bwd_expand(Seqs S, Groups GR, const double *__restrict__ phiT,
                                                    const double *__restrict__ qbuf,
                                                    const double *__restrict__ ginc, double *__restrict__ yend,
                                                    double *__restrict__ grad_zi) {
    constexpr int MM = M * M;
    __shared__ __attribute__((aligned(16))) double lds[CPW * (MM + M)];
    const int64_t gid = blockIdx.x;
    if (gid >= GR.ngroups) return;
    int64_t b, g;
    group_at(S, GR, gid, b, g);
    const SeqView sv = seq_view(S, b);
    if (g >= groups_of(sv.C, CPW)) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t c0 = g * CPW;
    const int nk = (int)min((int64_t)CPW, sv.C - c0);
    const bool need_first = (g == 0) && grad_zi;  // y(0) is dL/dzi
    stage_doubles(lds, phiT + (sv.cbase + c0) * MM, (int64_t)nk * MM, tid, blockDim.x);
    stage_doubles(lds + CPW * MM, qbuf + (sv.cbase + c0) * M, (int64_t)nk * M, tid, blockDim.x);
    double x = (tid < M) ? ginc[gid * M + tid] : 0.0;
    __syncthreads();
    if (tid >= 64) return;
    for (int k = nk - 1; k >= 0; --k) {
        const int64_t c = c0 + k;
        if (lane < M) yend[(sv.cbase + c) * M + lane] = x;
        if (k == 0 && !need_first) break;  // y at the group start is not needed
        const double q = lds[CPW * MM + k * M + (lane < M ? lane : 0)];
        if (c == sv.C - 1)  // the sequence's last chunk: y = q
            x = q;
        else
            x = reg_step<M>(lds + k * MM, M, 1, x, q, lane);
    }
    if (need_first && lane < M) grad_zi[b * M + lane] = x;
}

// ---------------------------------------------------------------- fused forward carry (grouped mode)
//
// One launch in place of a chain and an expansion: one block per group.  A
// block first forms its group's entry state by applying the maps of the groups
// before it (groups 0 .. g-1, from zi), then expands it through the group's own
// chunk transitions.  The prefix is recomputed by every block (at most n-1
// small matrix-vector products), so no block waits on another.  Maps and
// transitions are staged into LDS by all four waves; wave 0 applies them.
// (The same fusion of the adjoint carry was measured slower overall: the
// adjoint emit that follows it ran about 20 % longer.)

template <int M, int CPW>
struct FusedCarryShape {
    static constexpr int MM = M * M;
    // maps (with offsets) per staged batch, about 32 KiB, and at least a group's
    // transitions
    static constexpr int FIT = 4096 / (MM + M) > 0 ? 4096 / (MM + M) : 1;
    static constexpr int NBM = (FIT < 8 ? FIT : 8) > CPW ? (FIT < 8 ? FIT : 8) : CPW;
    static constexpr int BUF = NBM * (MM + M);
};

template <int M, int CPW>
__global__ __launch_bounds__(256) void k_fwd_carry(Seqs S, Groups GR, const double *__restrict__ zi,
                                                   const double *__restrict__ phiT,
                                                   const double *__restrict__ zbuf,
                                                   const double *__restrict__ aggbuf, double *__restrict__ xs,
                                                   uint32_t *__restrict__ nonfinite) {
    using FS = FusedCarryShape<M, CPW>;
    constexpr int MM = M * M;
    static_assert(CPW <= FS::NBM, "a group's transitions must fit one staged batch");
    __shared__ __attribute__((aligned(16))) double lds[FS::BUF];
    const int64_t gid = blockIdx.x;
    // the forward emit sets the flags; block gid clears sequence gid's (every
    // launch has at least one group slot per sequence)
    if (nonfinite && gid < S.n && threadIdx.x == 0) nonfinite[gid] = 0u;
    if (gid >= GR.ngroups) return;
    int64_t b, g;
    group_at(S, GR, gid, b, g);
    const SeqView sv = seq_view(S, b);
    if (g >= groups_of(sv.C, CPW)) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t gid0 = group_id(S, GR, b, 0);
    double x = (tid < M && zi) ? zi[b * M + tid] : 0.0;
    // x(g) = P_{g-1} ... P_0 zi + ... : the maps of the groups before g, in batches
    for (int64_t k0 = 0; k0 < g; k0 += FS::NBM) {
        const int nb = (int)min((int64_t)FS::NBM, g - k0);
        __syncthreads();
        stage_doubles(lds, aggbuf + (gid0 + k0) * (MM + M), (int64_t)nb * (MM + M), tid, blockDim.x);
        __syncthreads();
        if (tid < 64) {
            for (int k = 0; k < nb; ++k) {
                const double *A = lds + k * (MM + M);  // column-major map, then its offset
                x = reg_step<M>(A, 1, M, x, A[MM + (lane < M ? lane : 0)], lane);
            }
        }
    }
    // the group's chunks: x(c+1) = Phi_c x(c) + z_c
    const int64_t c0 = g * CPW;
    const int nk = (int)min((int64_t)CPW, sv.C - c0);
    const int nt = nk - 1;
    __syncthreads();
    stage_doubles(lds, phiT + (sv.cbase + c0) * MM, (int64_t)nt * MM, tid, blockDim.x);
    stage_doubles(lds + FS::NBM * MM, zbuf + (sv.cbase + c0) * M, (int64_t)nt * M, tid, blockDim.x);
    __syncthreads();
    if (tid >= 64) return;
    for (int k = 0; k < nk; ++k) {
        if (lane < M) xs[(sv.cbase + c0 + k) * M + lane] = x;
        if (k < nt) x = reg_step<M>(lds + k * MM, 1, M, x, lds[FS::NBM * MM + k * M + (lane < M ? lane : 0)], lane);
    }
}

}  // namespace tvlp
