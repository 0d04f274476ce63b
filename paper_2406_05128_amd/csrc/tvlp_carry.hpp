// Carries across chunks (gfx950).
//
// Group maps.  k_compose forms, for every group of consecutive chunks, the
// product of its chunks' affine maps (forward P_g, r_g; adjoint Psi_g, w_g),
// from the transitions and offsets the local scans stored.
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
// in flight; in the chain kernels seven waves stage the next batch while the
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

// ---------------------------------------------------------------- group maps
//
// A chunk's affine map is held as an M x (M+1) augmented matrix [A | v]
// (column-major, the offset v as column M, the implicit last row (0 ... 0 1)),
// so that one matrix product composes both parts: [A | v] [B | u] =
// [A B | A u + v].  Forward factors [Phi_c | z_c] (x(c+1) = Phi_c x(c) + z_c),
// multiplied later-on-the-left: [P_g | r_g] = F_{n-1} ... F_0.  Adjoint
// factors [Phi_c^T | q_c] (y(c) = Phi_c^T y(c+1) + q_c; Phi^T = 0 for the
// sequence's last chunk), earlier-on-the-left: [Psi_g | w_g] = F_0 ... F_{n-1}.
// The factors are multiplied as a binary tree (neighbour pairs, then pairs of
// pairs), one product per wave, so a group of n chunks takes ceil(log2 n)
// dependent products instead of n - 1.

template <int M>
struct ComposeShape {
    static constexpr int AUG = M * (M + 1);  // doubles per augmented matrix
    static constexpr int THREADS = 256;
    static constexpr int WAVES = THREADS / 64;
    // a wave's lanes as an 8 x 8 grid; lane (rt, ct) forms the outputs in rows
    // rt + 8r (r < RB) and columns ct + 8c (c < CB)
    static constexpr int RB = (M + 7) / 8;
    static constexpr int CB = (M + 1 + 7) / 8;
};

// C = X Y for augmented matrices in LDS, as a sum of M outer products; one
// wave, lane (rt, ct)'s outputs into registers.  Rows and columns past the
// matrix read a valid element and are never stored.
template <int M>
__device__ __forceinline__ void aug_product(const double *X, const double *Y,
                                            double (&acc)[ComposeShape<M>::RB][ComposeShape<M>::CB], int lane) {
    using CS = ComposeShape<M>;
    const int rt = lane >> 3, ct = lane & 7;
    int row[CS::RB], col[CS::CB];
#pragma unroll
    for (int r = 0; r < CS::RB; ++r) row[r] = min(rt + 8 * r, M - 1);
#pragma unroll
    for (int c = 0; c < CS::CB; ++c) col[c] = min(ct + 8 * c, M);
#pragma unroll
    for (int r = 0; r < CS::RB; ++r) {
        const double xo = X[M * M + row[r]];  // offset column: C[:, M] = X Y[:, M] + X[:, M]
#pragma unroll
        for (int c = 0; c < CS::CB; ++c) acc[r][c] = (col[c] == M) ? xo : 0.0;
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        double xv[CS::RB], yv[CS::CB];
#pragma unroll
        for (int r = 0; r < CS::RB; ++r) xv[r] = X[m * M + row[r]];
#pragma unroll
        for (int c = 0; c < CS::CB; ++c) yv[c] = Y[col[c] * M + m];
#pragma unroll
        for (int r = 0; r < CS::RB; ++r)
#pragma unroll
            for (int c = 0; c < CS::CB; ++c) acc[r][c] = fma(xv[r], yv[c], acc[r][c]);
    }
}

template <int M>
__device__ __forceinline__ void aug_store(double *C, const double (&acc)[ComposeShape<M>::RB][ComposeShape<M>::CB],
                                          int lane) {
    using CS = ComposeShape<M>;
    const int rt = lane >> 3, ct = lane & 7;
#pragma unroll
    for (int r = 0; r < CS::RB; ++r)
#pragma unroll
        for (int c = 0; c < CS::CB; ++c) {
            const int i = rt + 8 * r, j = ct + 8 * c;
            if (i < M && j <= M) C[j * M + i] = acc[r][c];
        }
}

// LDS of k_compose: the group's factors, multiplied in place.
template <int M>
constexpr size_t compose_lds_bytes(int cpw) { return (size_t)cpw * ComposeShape<M>::AUG * sizeof(double); }

// One block per group: forward (BWD false) [P_g | r_g] for every group but each
// sequence's last, written as aggbuf[gid] = P (column-major) then r; adjoint
// (BWD true) [Psi_g | w_g] for every group but each sequence's first, written as
// Psi (row-major) then w.  vec is zbuf (forward) or qbuf (adjoint).  Dynamic
// LDS: compose_lds_bytes<M>(CPW).
template <int M, int CPW, bool BWD>
__global__ __launch_bounds__(256) void k_compose(Seqs S, Groups GR, const double *__restrict__ phiT,
                                                 const double *__restrict__ vec, double *__restrict__ aggbuf) {
    using CS = ComposeShape<M>;
    constexpr int MM = M * M, AUG = CS::AUG;
    extern __shared__ __attribute__((aligned(16))) double fa[];  // [CPW][AUG]
    const int64_t gid = blockIdx.x;
    if (gid >= GR.ngroups) return;
    int64_t b, g;
    group_at(S, GR, gid, b, g);
    const SeqView sv = seq_view(S, b);
    const int64_t ng = groups_of(sv.C, CPW);
    if (g >= ng) return;
    if (BWD ? g == 0 : g == ng - 1) return;  // no map needed
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t c0 = g * CPW;
    const int n = (int)min((int64_t)CPW, sv.C - c0);
    const int64_t cb = sv.cbase + c0;
    // the factors: matrix part, then offsets; every load of a thread is issued
    // before its LDS writes (one memory latency for the whole staging)
    constexpr int NL = (CPW * MM + CS::THREADS - 1) / CS::THREADS;
    constexpr int NV = (CPW * M + CS::THREADS - 1) / CS::THREADS;
    double v[NL], u[NV];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int idx = tid + q * CS::THREADS;
        v[q] = 0.0;
        // adjoint: the sequence's last chunk has no transition (Phi^T = 0)
        if (idx < n * MM && (!BWD || c0 + idx / MM < sv.C - 1)) v[q] = phiT[cb * MM + idx];
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const int idx = tid + q * CS::THREADS;
        u[q] = idx < n * M ? vec[cb * M + idx] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int idx = tid + q * CS::THREADS;
        if (idx < n * MM) {
            const int k = idx / MM, r = idx - k * MM;
            if (!BWD) {
                fa[k * AUG + r] = v[q];
            } else {
                // phiT holds Phi column-major, i.e. Phi^T row-major: element
                // r = (i, j) of Phi^T goes to column j, row i
                const int i = r / M, j = r - i * M;
                fa[k * AUG + j * M + i] = v[q];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const int idx = tid + q * CS::THREADS;
        if (idx < n * M) {
            const int k = idx / M;
            fa[k * AUG + MM + (idx - k * M)] = u[q];
        }
    }
    __syncthreads();
    // level by level, in place: product p of a level (factors 2p, 2p+1) goes to
    // slot p once every product of its round has read its factors; slot p is
    // below every factor a later round reads
    int cnt = n;
    while (cnt > 1) {
        const int np = cnt / 2;
        for (int p0 = 0; p0 < np; p0 += CS::WAVES) {
            const int p = p0 + wv;
            double out[CS::RB][CS::CB];
            if (p < np) {
                const double *lo = fa + 2 * p * AUG, *hi = lo + AUG;
                aug_product<M>(BWD ? lo : hi, BWD ? hi : lo, out, lane);
            }
            __syncthreads();
            if (p < np) aug_store<M>(fa + p * AUG, out, lane);
            __syncthreads();
        }
        if (cnt & 1) {  // the odd factor moves up unchanged (slot np < cnt - 1)
            for (int idx = tid; idx < AUG; idx += CS::THREADS) fa[np * AUG + idx] = fa[(cnt - 1) * AUG + idx];
            __syncthreads();
        }
        cnt = np + (cnt & 1);
    }
    double *ag = aggbuf + gid * (MM + M);
    for (int idx = tid; idx < MM; idx += CS::THREADS) {
        if (!BWD) {
            ag[idx] = fa[idx];
        } else {  // row-major Psi: element idx = (i, j) from column j, row i
            const int i = idx / M, j = idx - i * M;
            ag[idx] = fa[j * M + i];
        }
    }
    for (int idx = tid; idx < M; idx += CS::THREADS) ag[MM + idx] = fa[MM + idx];
}

// One chunk per sequence (uniform batches with T <= L, such as frames filtered
// one by one): no chunk carries a transition, so the carries reduce to the
// state at the only chunk's boundary, st[b] = zi[b] (forward entry state) or
// zero (adjoint terminal state, zi null), and to clearing the per-sequence
// flags that the emits set, as the carry kernels do.  n sequences of M values.
template <int M>
__global__ __launch_bounds__(256) void k_single_chunk_states(int64_t n, const double *__restrict__ zi,
                                                             double *__restrict__ st,
                                                             uint32_t *__restrict__ nonfinite) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n * M) st[idx] = zi ? zi[idx] : 0.0;
    if (nonfinite && idx < n) nonfinite[idx] = 0u;
}

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
    if (wv == 0) __builtin_amdgcn_s_setprio(2);  // the serial wave issues ahead of the staging waves
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
    if (wv == 0) __builtin_amdgcn_s_setprio(2);  // the serial wave issues ahead of the staging waves
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
