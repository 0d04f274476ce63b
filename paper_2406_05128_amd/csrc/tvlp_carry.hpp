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
// first wave runs the current one.  The carried vector lives in LDS and every
// matrix row is one lane's dot product.
#pragma once

#include "tvlp_scan.hpp"

namespace tvlp {

// Orders this wave's memory operations for the compiler (a wavefront-scope
// fence, so values other lanes wrote to LDS are read again, not reused) and
// keeps the scheduler from moving instructions across.  LDS operations of one
// wave are executed in order, so no hardware wait is needed between lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Copies n doubles from global to LDS; thread t of nt cooperating threads.
// Sixteen loads per thread are issued before their LDS writes, so a batch pays
// about one memory latency per sixteen rounds instead of one per element.
__device__ __forceinline__ void stage_doubles(double *dst, const double *__restrict__ src, int64_t n, int t, int nt) {
    constexpr int U = 16;
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

// v <- A v + z for the M-vector v in LDS; A[i][j] = A_[i * si + j * sj] in LDS,
// z held by lane i.  One wave; lane i < M computes row i; every lane's reads
// of v precede the write of the new v.
template <int M>
__device__ __forceinline__ void lds_step(const double *A_, int si, int sj, double *v, double z, int lane) {
    const int i = lane < M ? lane : 0;
    double acc0 = z, acc1 = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const double aij = A_[i * si + j * sj];
        if (j & 1)
            acc1 = fma(aij, v[j], acc1);
        else
            acc0 = fma(aij, v[j], acc0);
    }
    wave_sync();
    if (lane < M) v[lane] = acc0 + acc1;
    wave_sync();
}

// v <- z (lane i < M holds z_i).
template <int M>
__device__ __forceinline__ void lds_set(double *v, double z, int lane) {
    wave_sync();
    if (lane < M) v[lane] = z;
    wave_sync();
}

template <int M>
struct CarryShape {
    static constexpr int MM = M * M;
    static constexpr int THREADS = 256;         // chain and expand kernels: four waves
    static constexpr int BUF_DOUBLES = 8000;    // one chain-kernel staging buffer (62.5 KiB)
    // matrices (each with its offset vector) per chain-kernel batch
    static constexpr int NB = BUF_DOUBLES / (MM + M) > 0 ? BUF_DOUBLES / (MM + M) : 1;
};

// ---------------------------------------------------------------- forward

// Chained: items are chunks (matrix Phi_c, offset z_c; output xs per chunk);
// grouped: items are groups (map with its offset; output ginc per group).
// The last item has no map.
template <int M>
__global__ __launch_bounds__(256) void k_fwd_chain(Seqs S, Groups GR, const double *__restrict__ zi,
                                                   const double *__restrict__ phiT,
                                                   const double *__restrict__ zbuf,
                                                   const double *__restrict__ aggbuf, double *__restrict__ ginc,
                                                   double *__restrict__ xs, int chain,
                                                   uint32_t *__restrict__ nonfinite) {
    using CS = CarryShape<M>;
    constexpr int MM = M * M;
    __shared__ double lds[2 * CS::BUF_DOUBLES + M];
    double *v = lds + 2 * CS::BUF_DOUBLES;
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
    if (wv == 0 && lane < M) v[lane] = zi ? zi[b * M + lane] : 0.0;
    stage(0, tid, CS::THREADS);
    __syncthreads();
    for (int64_t bi = 0; bi < nbatch; ++bi) {
        if (wv == 0) {
            const double *buf = lds + (bi & 1) * CS::BUF_DOUBLES;
            const int64_t k0 = bi * CS::NB;
            const int nb = (int)min((int64_t)CS::NB, n - k0);
            for (int k = 0; k < nb; ++k) {
                if (lane < M) out[(id0 + k0 + k) * M + lane] = v[lane];
                if (k0 + k + 1 < n) {
                    const double *A = chain ? buf + k * MM : buf + k * (MM + M);
                    const double *z = chain ? buf + CS::NB * MM + k * M : A + MM;
                    lds_step<M>(A, 1, M, v, lane < M ? z[lane] : 0.0, lane);
                }
            }
        } else if (bi + 1 < nbatch) {
            stage(bi + 1, tid - 64, CS::THREADS - 64);
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
__global__ __launch_bounds__(256) void k_bwd_chain(Seqs S, Groups GR, const double *__restrict__ phiT,
                                                   const double *__restrict__ qbuf,
                                                   const double *__restrict__ aggbuf, double *__restrict__ ginc,
                                                   double *__restrict__ yend, double *__restrict__ grad_zi,
                                                   int chain, uint32_t *__restrict__ nonfinite) {
    using CS = CarryShape<M>;
    constexpr int MM = M * M;
    __shared__ double lds[2 * CS::BUF_DOUBLES + M];
    double *v = lds + 2 * CS::BUF_DOUBLES;
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
    if (wv == 0 && lane < M) v[lane] = 0.0;
    stage(0, tid, CS::THREADS);
    __syncthreads();
    for (int64_t bi = 0; bi < nbatch; ++bi) {
        if (wv == 0) {
            const double *buf = lds + (bi & 1) * CS::BUF_DOUBLES;
            int64_t k0;
            int nb;
            range(bi, k0, nb);
            for (int k = nb - 1; k >= 0; --k) {
                const int64_t item = k0 + k;
                if (lane < M) out[(id0 + item) * M + lane] = v[lane];
                if (chain) {
                    const double q = lane < M ? buf[CS::NB * MM + k * M + lane] : 0.0;
                    if (item == n - 1)
                        lds_set<M>(v, q, lane);
                    else
                        lds_step<M>(buf + k * MM, M, 1, v, q, lane);
                } else if (item > 0) {
                    const double *A = buf + k * (MM + M);
                    lds_step<M>(A, M, 1, v, lane < M ? A[MM + lane] : 0.0, lane);
                }
            }
            if (chain && bi + 1 == nbatch && grad_zi && lane < M) grad_zi[b * M + lane] = v[lane];
        } else if (bi + 1 < nbatch) {
            stage(bi + 1, tid - 64, CS::THREADS - 64);
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
    __shared__ double lds[CPW * (MM + M) + M];
    double *v = lds + CPW * (MM + M);
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
    if (tid < M) v[tid] = ginc[gid * M + tid];
    __syncthreads();
    if (tid >= 64) return;
    for (int k = nk - 1; k >= 0; --k) {
        const int64_t c = c0 + k;
        if (lane < M) yend[(sv.cbase + c) * M + lane] = v[lane];
        if (k == 0 && !need_first) break;  // y at the group start is not needed
        const double q = lane < M ? lds[CPW * MM + k * M + lane] : 0.0;
        if (c == sv.C - 1)  // the sequence's last chunk: y = q
            lds_set<M>(v, q, lane);
        else
            lds_step<M>(lds + k * MM, M, 1, v, q, lane);
    }
    if (need_first && lane < M) grad_zi[b * M + lane] = v[lane];
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
    __shared__ double lds[FS::BUF + M];
    double *v = lds + FS::BUF;
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
    if (tid < M) v[tid] = zi ? zi[b * M + tid] : 0.0;
    // x(g) = P_{g-1} ... P_0 zi + ... : the maps of the groups before g, in batches
    for (int64_t k0 = 0; k0 < g; k0 += FS::NBM) {
        const int nb = (int)min((int64_t)FS::NBM, g - k0);
        __syncthreads();
        stage_doubles(lds, aggbuf + (gid0 + k0) * (MM + M), (int64_t)nb * (MM + M), tid, blockDim.x);
        __syncthreads();
        if (tid < 64) {
            for (int k = 0; k < nb; ++k) {
                const double *A = lds + k * (MM + M);  // column-major map, then its offset
                lds_step<M>(A, 1, M, v, lane < M ? A[MM + lane] : 0.0, lane);
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
        if (lane < M) xs[(sv.cbase + c0 + k) * M + lane] = v[lane];
        if (k < nt) lds_step<M>(lds + k * MM, 1, M, v, lane < M ? lds[FS::NBM * MM + k * M + lane] : 0.0, lane);
    }
}

}  // namespace tvlp
