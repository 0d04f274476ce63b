// Host side of the C ABI declared in include/tvlp.h: plans, argument checks,
// workspace management and kernel dispatch over the compiled filter orders.
#include "tvlp.h"
#include "tvlp_ops.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace tvlp;
using namespace tvlp_host;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace

// Error reporting shared with the other translation units of the library.
namespace tvlp_host {
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }
}  // namespace tvlp_host

namespace {

int check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return LP_OK;
    return fail(LP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = (prev == dev) || hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

constexpr int kOrders[] = {1, 2, 3, 4, 6, 8, 10, 12, 16, 20, 22, 24, 32};

bool order_supported(int M) {
    for (int m : kOrders)
        if (m == M) return true;
    return false;
}

// shortest chunk length the autotuner considers for LP_FLAG_HIGH_RADIUS plans
constexpr int kAccurateChunk = 1536;

int default_chunk(int M) {
    int mult = (256 + M - 1) / M;
    return std::max(1, mult) * M;
}


// Lanes per chunk and columns per lane of the basis pass for order M.
template <int M>
struct BasisShape {
    static constexpr int LPC = M >= 8 ? 8 : (M >= 2 ? 4 : 2);
    static constexpr int CPL = (M + 1 + LPC - 1) / LPC;
};

struct Launch {
    hipStream_t stream;
};

// Bytes of the various per-chunk arrays (float64).
size_t bytes_state(int M, int64_t nch) { return (size_t)nch * M * sizeof(double); }
size_t bytes_phi(int M, int64_t nch) { return (size_t)nch * M * M * sizeof(double); }

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr size_t kStatusOffset = 256;  // byte offset of the scan status word in every workspace

// Workspace layout for one call with nch chunks and n samples over B sequences.
struct WsLayout {
    size_t zero, xs, phi, yend, q, cbase, gbf, gbb, aggf, inclf, aggb, inclb, sbuf, fpart, status, total;
};

// ngf / ngb: group slots of the forward / adjoint scans; nsamp: sample slots
// of the sequence layout (B*T, or N), for s recomputed by the adjoint;
// fpart_bytes: the chunks' shares of a frame-rate coefficient gradient.
// fwd_only: the forward's regions only (the adjoint's q, group maps, recomputed s
// and frame shares get no space).
WsLayout ws_layout(int M, int64_t nch, int64_t B, int64_t ngf, int64_t ngb, int64_t nsamp,
                   size_t fpart_bytes = 0, bool fwd_only = false) {
    if (fwd_only) {
        ngb = 0;
        nsamp = 0;
        fpart_bytes = 0;
    }
    WsLayout w{};
    size_t off = 0;
    const size_t agg = (size_t)(M * M + M) * sizeof(double);
    w.zero = off;  off += 256;   // stays zero (the ring DMAs' spare lanes read it)
    w.status = off;  off += 256;  // status word at a fixed offset
    w.xs = off;    off += align_up(bytes_state(M, nch));
    w.phi = off;   off += align_up(bytes_phi(M, nch));
    w.yend = off;  off += align_up(bytes_state(M, nch));  // adjoint: yend; forward: z of every chunk
    w.q = off;     off += fwd_only ? 0 : align_up(bytes_state(M, nch));
    w.cbase = off; off += align_up((size_t)(B + 1) * sizeof(int64_t));
    w.gbf = off;   off += align_up((size_t)(B + 1) * sizeof(int64_t));
    w.gbb = off;   off += align_up((size_t)(B + 1) * sizeof(int64_t));
    w.aggf = off;  off += align_up((size_t)ngf * agg);
    w.inclf = off; off += align_up((size_t)ngf * M * sizeof(double));
    w.aggb = off;  off += align_up((size_t)ngb * agg);
    w.inclb = off; off += align_up((size_t)ngb * M * sizeof(double));
    w.sbuf = off;  off += align_up((size_t)nsamp * sizeof(float));
    w.fpart = off; off += align_up(fpart_bytes);
    w.total = off;
    return w;
}

int ensure_ws(lp_plan *p, size_t need, hipStream_t stream) {
    if (p->ws_bytes >= need) return LP_OK;
    if (p->live_graphs > 0)
        return fail(LP_EINVAL,
                    "workspace of %zu bytes needed but %d captured graph(s) hold the current one (%zu bytes); "
                    "destroy them first or reserve a larger workspace before capturing",
                    need, p->live_graphs, p->ws_bytes);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (stream && hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(LP_ENOMEM, "workspace of %zu bytes needed during graph capture; call lp_plan_reserve first", need);
    if (p->ws) {
        // the previous workspace may still be in use by queued work
        if (hipDeviceSynchronize() != hipSuccess) return fail(LP_EDEVICE, "device sync before workspace growth failed");
        (void)hipFree(p->ws);
        p->ws = nullptr;
        p->ws_bytes = 0;
    }
    void *ptr = nullptr;
    if (hipMalloc(&ptr, need) != hipSuccess) return fail(LP_ENOMEM, "hipMalloc(%zu) for the workspace failed", need);
    if (hipMemset(ptr, 0, kStatusOffset + 256) != hipSuccess) {
        (void)hipFree(ptr);
        return fail(LP_EDEVICE, "workspace initialisation failed");
    }
    p->ws = ptr;
    p->ws_bytes = need;
    return LP_OK;
}

// ---------------------------------------------------------------- static scratch
// The no-allocation forward (lp_forward_noalloc) takes its workspace from this
// array instead of the plan's allocation.  Host code must not pass `scratch`
// itself to a kernel (in host code it names a host-side stand-in): its device
// address is looked up once per device with hipGetSymbolAddress and kept in
// g_scratch.
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];

__global__ void k_zero_words(uint32_t *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// Device address of this device's scratch (the current device must be `device`);
// the first call per device looks it up and clears the zero block and status
// word at its head (a fill kernel, then a device synchronisation).
int scratch_of(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return fail(LP_EINVAL, "device %d beyond the scratch table", device);
    if (!g_scratch[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return fail(LP_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d", device);
        hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, nullptr, (uint32_t *)ptr,
                           (int)((kStatusOffset + 256) / 4));
        if (int r = check_hip(hipGetLastError(), "scratch clear launch")) return r;
        if (int r = check_hip(hipDeviceSynchronize(), "scratch clear")) return r;
        g_scratch[device] = ptr;
    }
    *out = g_scratch[device];
    return LP_OK;
}

// ---------------------------------------------------------------- frame-wise approximation
// Frames of length W = 4 hop, frame f starting at sample (f - 3) hop, F =
// ceil(T / hop) + 3 per sequence: every sample lies in exactly four frames.
// The optional weight is w(n) / 2 with the periodic Hann window w(n) =
// sin^2(pi n / W), whose shifted copies sum to 2 at this overlap.
__device__ __forceinline__ float frame_weight(int64_t n, int64_t W) {
    const float sn = sinpif((float)n / (float)W);
    return 0.5f * sn * sn;
}

// xf[b][f][n] = x[b][(f - 3) hop + n] (0 outside the signal), times the weight if asked.
__global__ __launch_bounds__(256) void k_frames_gather(int64_t B, int64_t T, int64_t hop, int64_t F,
                                                       const float *__restrict__ x, float *__restrict__ xf,
                                                       int weighted) {
    const int64_t W = 4 * hop, n_all = B * F * W;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_all;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t n = q % W, bf = q / W, f = bf % F, b = bf / F;
        const int64_t t = (f - 3) * hop + n;
        float v = (t >= 0 && t < T) ? x[b * T + t] : 0.f;
        if (weighted) v *= frame_weight(n, W);
        xf[q] = v;
    }
}

// x[b][t] = sum over the four frames holding t of xf[b][f][t - (f - 3) hop], each
// times the weight if asked (the adjoint of k_frames_gather).
__global__ __launch_bounds__(256) void k_frames_overlap_add(int64_t B, int64_t T, int64_t hop, int64_t F,
                                                            const float *__restrict__ xf, float *__restrict__ x,
                                                            int weighted) {
    const int64_t W = 4 * hop, n_all = B * T;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_all;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = q % T, b = q / T, f0 = t / hop;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t f = f0 + j, n = t - (f - 3) * hop;
            const float v = xf[(b * F + f) * W + n];
            acc += (double)(weighted ? frame_weight(n, W) * v : v);
        }
        x[q] = (float)acc;
    }
}

// Prefix sums over a sequence table (single block): chunk counts (cbase) and
// the group counts of the forward (gbf, cpwf chunks per group) and adjoint
// (gbb, cpwb) scans.  The table is either packed offsets or starts + lens;
// lengths are clamped exactly as seq_view clamps them.
__global__ __launch_bounds__(1024) void k_build_tables(const int64_t *__restrict__ offsets,
                                                       const int64_t *__restrict__ starts,
                                                       const int64_t *__restrict__ lens, int64_t n, int L,
                                                       int64_t N, int cpwf, int cpwb, int64_t nch_cap,
                                                       int64_t *__restrict__ cbase, int64_t *__restrict__ gbf,
                                                       int64_t *__restrict__ gbb, int *__restrict__ status) {
    __shared__ int64_t part[3][1024];
    __shared__ int64_t carry[3];
    if (threadIdx.x < 3) carry[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += 1024) {
        const int64_t b = base + threadIdx.x;
        int64_t cnt = 0;
        if (b < n) {
            int64_t lo, hi;
            if (offsets) {
                lo = min(max(offsets[b], (int64_t)0), N);
                hi = min(max(offsets[b + 1], lo), N);
            } else {
                lo = min(max(starts[b], (int64_t)0), N);
                hi = min(max(lo + lens[b], lo), N);
            }
            const int64_t len = hi - lo;
            cnt = len <= 0 ? 0 : (len + L - 1) / L;
        }
        part[0][threadIdx.x] = cnt;
        part[1][threadIdx.x] = (cnt + cpwf - 1) / cpwf;
        part[2][threadIdx.x] = (cnt + cpwb - 1) / cpwb;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            int64_t v0 = 0, v1 = 0, v2 = 0;
            if (threadIdx.x >= (unsigned)d) {
                v0 = part[0][threadIdx.x - d];
                v1 = part[1][threadIdx.x - d];
                v2 = part[2][threadIdx.x - d];
            }
            __syncthreads();
            part[0][threadIdx.x] += v0;
            part[1][threadIdx.x] += v1;
            part[2][threadIdx.x] += v2;
            __syncthreads();
        }
        if (b < n) {
            cbase[b + 1] = carry[0] + part[0][threadIdx.x];
            gbf[b + 1] = carry[1] + part[1][threadIdx.x];
            gbb[b + 1] = carry[2] + part[2][threadIdx.x];
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            carry[0] += part[0][1023];
            carry[1] += part[1][1023];
            carry[2] += part[2][1023];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cbase[0] = 0;
        gbf[0] = 0;
        gbb[0] = 0;
        // more chunks than the launch was sized for: the excess is not computed
        if (carry[0] > nch_cap) atomicOr(status, 2);
    }
}

// y = s0 + s1 for a stacked filter pair (n samples each); vec: y, s2 and
// s2 + n are 16-byte aligned.
__global__ __launch_bounds__(256) void k_pair_sum(float *__restrict__ y, const float *__restrict__ s2, int64_t n,
                                                  int vec) {
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (vec && i0 + 3 < n) {
        const float4 u = *reinterpret_cast<const float4 *>(s2 + i0);
        const float4 v = *reinterpret_cast<const float4 *>(s2 + n + i0);
        *reinterpret_cast<float4 *>(y + i0) = make_float4(u.x + v.x, u.y + v.y, u.z + v.z, u.w + v.w);
    } else {
        const int64_t i1 = i0 + 4 < n ? i0 + 4 : n;
        for (int64_t i = i0; i < i1; ++i) y[i] = s2[i] + s2[n + i];
    }
}

// Deterministic stand-in values for the autotuner's timed runs: x[i] = scale * u
// with u in [-1, 1) from a 32-bit integer mix of (i, seed) (xorshift-multiply
// rounds).  The kernels' time depends on the values they see (their power draw
// and hence the clock), so the candidates are timed on data rather than zeros.
__global__ __launch_bounds__(256) void k_tune_fill(float *__restrict__ x, int64_t n, float scale, uint32_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i ^ (uint32_t)(i >> 32) * 0x9e3779b9u ^ seed;
        h ^= h >> 16;
        h *= 0x7feb352du;
        h ^= h >> 15;
        h *= 0x846ca68bu;
        h ^= h >> 16;
        x[i] = scale * ((float)(h >> 8) * (1.0f / 8388608.0f) - 1.0f);
    }
}

// Forward / adjoint scan group sizes (chunks per wave) of order M.
int scan_cpw(int M, bool fwd) {
    int r = 0;
    auto pick = [&](auto ops) {
        using O = decltype(ops);
        r = fwd ? O::FS::CPW : O::RS::CPW;
    };
    switch (M) {
#define TVLP_CPW(m) \
    case m:         \
        pick(Ops<m>{}); \
        break;
        TVLP_CPW(1) TVLP_CPW(2) TVLP_CPW(3) TVLP_CPW(4) TVLP_CPW(6) TVLP_CPW(8) TVLP_CPW(10)
        TVLP_CPW(12) TVLP_CPW(16) TVLP_CPW(20) TVLP_CPW(22) TVLP_CPW(24) TVLP_CPW(32)
#undef TVLP_CPW
    default:
        r = 1;
    }
    return r;
}

template <class F>
bool dispatch(int M, F &&f) {
    switch (M) {
#define TVLP_CASE(m) \
    case m:          \
        f(Ops<m>{}); \
        return true;
        TVLP_CASE(1)
        TVLP_CASE(2)
        TVLP_CASE(3)
        TVLP_CASE(4)
        TVLP_CASE(6)
        TVLP_CASE(8)
        TVLP_CASE(10)
        TVLP_CASE(12)
        TVLP_CASE(16)
        TVLP_CASE(20)
        TVLP_CASE(22)
        TVLP_CASE(24)
        TVLP_CASE(32)
#undef TVLP_CASE
    default:
        return false;
    }
}

int check_plan(const lp_plan *p) {
    if (!p) return fail(LP_EINVAL, "plan is NULL");
    return LP_OK;
}

int64_t uniform_nchunks(int64_t B, int64_t T, int L) { return B * ceil_div(T, L); }

// Resolves sequence tables, group counts and workspace regions for one call.
// ws_ext: a forward-only call into this caller-provided workspace of ws_cap bytes
// (the static scratch) instead of the plan's own.
template <class O>
int prepare(lp_plan *p, int64_t B, const int64_t *offsets, int64_t T_or_N, const void *saved, hipStream_t st,
            typename O::Bufs &w, const int64_t *starts = nullptr, const int64_t *lens = nullptr,
            int64_t bound = 0, size_t fpart_bytes = 0, char *ws_ext = nullptr, size_t ws_cap = 0) {
    const int M = p->M, L = p->L;
    const int cpwf = O::FS::CPW, cpwb = O::RS::CPW;
    int64_t nch, ngf, ngb;
    const bool tabled = offsets || starts;
    if (tabled) {
        // non-overlapping sequences inside [0, N) hold at most N samples
        const int64_t tot = (bound > 0 && bound < T_or_N) ? bound : T_or_N;
        nch = ceil_div(tot, L) + B;
        ngf = ceil_div(nch, cpwf) + B;
        ngb = ceil_div(nch, cpwb) + B;
    } else {
        const int64_t C = ceil_div(T_or_N, L);
        nch = B * C;
        ngf = B * ceil_div(C, cpwf);
        ngb = B * ceil_div(C, cpwb);
    }
    WsLayout lay = ws_layout(M, nch, B, ngf, ngb, tabled ? T_or_N : B * T_or_N, fpart_bytes, ws_ext != nullptr);
    if (ws_ext) {
        if (lay.total > ws_cap)
            return fail(LP_EINVAL, "the call needs %zu bytes of scratch; the static scratch holds %zu", lay.total,
                        ws_cap);
    } else if (int r = ensure_ws(p, lay.total, st)) {
        return r;
    }
    char *ws = ws_ext ? ws_ext : (char *)p->ws;
    w.nch = nch;
    w.S = Seqs{nullptr, nullptr, nullptr, nullptr, tabled ? 0 : T_or_N, B, L, tabled ? T_or_N : 0, nch, 0};
    w.gf = Groups{nullptr, ngf, cpwf};
    w.gb = Groups{nullptr, ngb, cpwb};
    if (tabled) {
        int64_t *cb = (int64_t *)(ws + lay.cbase);
        int64_t *gbf = (int64_t *)(ws + lay.gbf);
        int64_t *gbb = (int64_t *)(ws + lay.gbb);
        hipLaunchKernelGGL(k_build_tables, dim3(1), dim3(1024), 0, st, offsets, starts, lens, B, L, T_or_N, cpwf,
                           cpwb, nch, cb, gbf, gbb, (int *)(ws + lay.status));
        w.S.offsets = offsets;
        w.S.starts = starts;
        w.S.lens = lens;
        w.S.cbase = cb;
        w.gf.gbase = gbf;
        w.gb.gbase = gbb;
    }
    if (saved) {
        w.xs = (double *)saved;
        w.phiT = (double *)((char *)saved + bytes_state(M, nch));
    } else {
        w.xs = (double *)(ws + lay.xs);
        w.phiT = (double *)(ws + lay.phi);
    }
    w.yend = (double *)(ws + lay.yend);
    w.zbuf = w.yend;  // the forward's chunk offsets share the adjoint's yend region
    w.qbuf = (double *)(ws + lay.q);
    w.aggf = (double *)(ws + lay.aggf);
    w.inclf = (double *)(ws + lay.inclf);
    w.aggb = (double *)(ws + lay.aggb);
    w.inclb = (double *)(ws + lay.inclb);
    w.status = (int *)(ws + lay.status);
    w.zero = (const float *)(ws + lay.zero);
    w.sbuf = (float *)(ws + lay.sbuf);
    w.fpart = (double *)(ws + lay.fpart);
    w.chain = (p->flags & LP_FLAG_CHAINED_CARRY) ? 1 : 0;
    w.nonfinite = nullptr;
    return LP_OK;
}

// Common driver of the uniform and varlen forward.
int forward_impl(lp_plan *p, int64_t B, const int64_t *offsets, int64_t T_or_N, const float *e, const float *a,
                 const double *zi, float *s, double *zf, void *saved, void *stream,
                 const int64_t *starts = nullptr, const int64_t *lens = nullptr, int64_t bound = 0,
                 bool ti = false, bool noalloc = false, uint32_t *nonfinite = nullptr) {
    if (int r = check_plan(p)) return r;
    if (B < 1) return fail(LP_EINVAL, "B must be >= 1 (got %lld)", (long long)B);
    if (T_or_N < 1) return fail(LP_EINVAL, "T (or N) must be >= 1 (got %lld)", (long long)T_or_N);
    if (!e || !a || !s) return fail(LP_EINVAL, "e, a and s are required");
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(LP_EDEVICE, "cannot select device %d", p->device);
    hipStream_t st = (hipStream_t)stream;
    int rc = LP_OK;
    void *sc = nullptr;
    if (noalloc) {
        if (!saved) return fail(LP_EINVAL, "the no-allocation forward needs a caller-provided saved buffer");
        if (int r = scratch_of(p->device, &sc)) return r;
    }
    // no timing events on the no-allocation path (event creation may allocate)
    Timer tm{noalloc ? nullptr : p, st};
    dispatch(p->M, [&](auto ops) {
        using O = decltype(ops);
        typename O::Bufs w;
        rc = prepare<O>(p, B, offsets, T_or_N, saved, st, w, starts, lens, bound, 0, (char *)sc,
                        noalloc ? kScratchBytes : 0);
        w.S.ti = ti ? 1 : 0;
        w.nonfinite = nonfinite;
        if (rc == LP_OK) O::forward(w, e, a, zi, s, zf, st, tm);
    });
    if (rc != LP_OK) return rc;
    return check_hip(hipGetLastError(), "kernel launch (forward)");
}

int backward_impl(lp_plan *p, int64_t B, const int64_t *offsets, int64_t T_or_N, const float *g, const float *a,
                  const float *e, const double *zi, const float *s, const void *saved, float *ge, float *ga,
                  double *gzi, void *stream, int64_t gshare = 0, bool ti = false, uint32_t *nonfinite = nullptr) {
    if (int r = check_plan(p)) return r;
    if (B < 1) return fail(LP_EINVAL, "B must be >= 1 (got %lld)", (long long)B);
    if (T_or_N < 1) return fail(LP_EINVAL, "T (or N) must be >= 1 (got %lld)", (long long)T_or_N);
    if (!g || !a || !saved) return fail(LP_EINVAL, "g, a and saved are required");
    if ((ga || ge) && !s && !e) return fail(LP_EINVAL, "the adjoint needs s or e (to recompute s)");
    if (!ge && !ga && !gzi && !nonfinite) return LP_OK;
    (void)zi;
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(LP_EDEVICE, "cannot select device %d", p->device);
    hipStream_t st = (hipStream_t)stream;
    int rc = LP_OK;
    Timer tm{p, st};
    dispatch(p->M, [&](auto ops) {
        using O = decltype(ops);
        typename O::Bufs w;
        rc = prepare<O>(p, B, offsets, T_or_N, saved, st, w);
        w.S.gshare = gshare;
        w.S.ti = ti ? 1 : 0;
        w.nonfinite = nonfinite;
        if (rc == LP_OK) O::backward(w, g, a, e, s, ge, ga, gzi, st, tm);
    });
    if (rc != LP_OK) return rc;
    return check_hip(hipGetLastError(), "kernel launch (backward)");
}

}  // namespace

extern "C" {

const char *lp_version(void) { return "tvlp 0.1 gfx950"; }

const char *lp_last_error(void) { return g_err.c_str(); }

int lp_supported_orders(int *out, int cap) {
    const int n = (int)(sizeof kOrders / sizeof kOrders[0]);
    if (out)
        for (int i = 0; i < n && i < cap; ++i) out[i] = kOrders[i];
    return n;
}

int lp_plan_create(lp_plan **out, int device, int M, int flags) {
    if (!out) return fail(LP_EINVAL, "out is NULL");
    *out = nullptr;
    if (M < 1 || M > 64) return fail(LP_EINVAL, "order M must be in [1, 64] (got %d)", M);
    if (!order_supported(M)) return fail(LP_EINVAL, "order M = %d has no compiled chunked kernels", M);
    if (flags & ~(LP_FLAG_CHAINED_CARRY | LP_FLAG_HIGH_RADIUS)) return fail(LP_EINVAL, "unknown plan flags 0x%x", flags);
    if (flags & LP_FLAG_HIGH_RADIUS) flags |= LP_FLAG_CHAINED_CARRY;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(LP_EINVAL, "device %d not available", device);
    lp_plan *p = new (std::nothrow) lp_plan{};
    if (!p) return fail(LP_ENOMEM, "out of host memory");
    p->device = device;
    p->M = M;
    p->L = default_chunk(M);
    if (flags & LP_FLAG_HIGH_RADIUS) dispatch(M, [&](auto ops) { p->L = decltype(ops)::max_chunk(); });
    p->flags = flags;
    p->carry_fixed = (flags & LP_FLAG_CHAINED_CARRY) != 0;
    {
        // the static scratch of the plan's device is looked up (and cleared) here,
        // ahead of any capture a caller of lp_forward_noalloc may start later
        DeviceGuard dg(device);
        void *sc = nullptr;
        const int r = dg.ok ? scratch_of(device, &sc) : fail(LP_EDEVICE, "cannot select device %d", device);
        if (r != LP_OK) {
            delete p;
            return r;
        }
    }
    *out = p;
    return LP_OK;
}

int lp_plan_destroy(lp_plan *p) {
    if (!p) return LP_OK;
    if (p->live_graphs > 0)
        return fail(LP_EINVAL, "plan still has %d captured graph(s); destroy them first", p->live_graphs);
    for (auto &r : p->pending) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    if (p->ws) {
        DeviceGuard dg(p->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(p->ws);
    }
    delete p;
    return LP_OK;
}

int lp_plan_set_chunk(lp_plan *p, int L) {
    if (int r = check_plan(p)) return r;
    if (L < p->M || L % p->M != 0) return fail(LP_EINVAL, "chunk length %d must be a positive multiple of M = %d", L, p->M);
    // the adjoint emit kernel keeps each of its chunks' s in LDS
    int maxL = 0;
    dispatch(p->M, [&](auto ops) { maxL = decltype(ops)::max_chunk(); });
    if (L > maxL) return fail(LP_EINVAL, "chunk length %d exceeds the maximum %d for M = %d", L, maxL, p->M);
    if (p->live_graphs > 0 && L != p->L)
        return fail(LP_EINVAL, "chunk length is fixed while %d captured graph(s) use the plan", p->live_graphs);
    p->L = L;
    return LP_OK;
}

int lp_plan_get_chunk(const lp_plan *p) { return p ? p->L : 0; }

int lp_plan_set_carry(lp_plan *p, int mode) {
    if (int r = check_plan(p)) return r;
    if (mode < -1 || mode > 1) return fail(LP_EINVAL, "carry mode must be -1, 0 or 1 (got %d)", mode);
    if (p->flags & LP_FLAG_HIGH_RADIUS) {
        if (mode != 1) return fail(LP_EINVAL, "a high-radius plan keeps the chained carry");
        return LP_OK;
    }
    if (mode < 0) {  // release: the autotuner chooses again
        p->carry_fixed = false;
        return LP_OK;
    }
    p->flags = mode ? (p->flags | LP_FLAG_CHAINED_CARRY) : (p->flags & ~LP_FLAG_CHAINED_CARRY);
    p->carry_fixed = true;
    return LP_OK;
}

int lp_plan_get_carry(const lp_plan *p) { return p ? ((p->flags & LP_FLAG_CHAINED_CARRY) ? 1 : 0) : -1; }

int lp_plan_set_timing(lp_plan *p, int on) {
    if (int r = check_plan(p)) return r;
    p->timing = on != 0;
    return LP_OK;
}

int lp_plan_timings(lp_plan *p, char *names, int name_len, double *ms, int64_t *launches, int cap) {
    if (int r = check_plan(p)) return r;
    DeviceGuard dg(p->device);
    for (auto &r : p->pending) {
        float t = 0.f;
        if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&t, r.start, r.stop) == hipSuccess) {
            auto &acc = p->totals[r.name];
            acc.first += t;
            acc.second += 1;
        }
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    p->pending.clear();
    int i = 0;
    for (auto &kv : p->totals) {
        if (i < cap) {
            if (names && name_len > 0) {
                std::strncpy(names + (size_t)i * name_len, kv.first.c_str(), (size_t)name_len - 1);
                names[(size_t)i * name_len + name_len - 1] = 0;
            }
            if (ms) ms[i] = kv.second.first;
            if (launches) launches[i] = kv.second.second;
        }
        ++i;
    }
    return i;
}

int lp_plan_status(lp_plan *p) {
    if (int r = check_plan(p)) return r;
    if (!p->ws) return LP_OK;
    DeviceGuard dg(p->device);
    if (hipDeviceSynchronize() != hipSuccess) return fail(LP_EDEVICE, "device error before status read");
    // the status word sits at a fixed offset from the end of the workspace layout
    int v = 0;
    if (hipMemcpy(&v, (char *)p->ws + kStatusOffset, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(LP_EDEVICE, "status read failed");
    if (v != 0) {
        const int zero = 0;
        (void)hipMemcpy((char *)p->ws + kStatusOffset, &zero, sizeof(int), hipMemcpyHostToDevice);
        return fail(LP_EINVAL, "segments held more samples than total_bound (status %d)", v);
    }
    return LP_OK;
}

int lp_plan_reset_timings(lp_plan *p) {
    if (int r = check_plan(p)) return r;
    (void)lp_plan_timings(p, nullptr, 0, nullptr, nullptr, 0);
    p->totals.clear();
    return LP_OK;
}

int lp_plan_reserve(lp_plan *p, int64_t B, int64_t T) {
    if (int r = check_plan(p)) return r;
    if (B < 1 || T < 1) return fail(LP_EINVAL, "B and T must be >= 1");
    DeviceGuard dg(p->device);
    const int64_t nch = uniform_nchunks(B, T, p->L) + B;
    const int cf = scan_cpw(p->M, true), cb = scan_cpw(p->M, false);
    WsLayout w = ws_layout(p->M, nch, B, ceil_div(nch, cf) + B, ceil_div(nch, cb) + B, B * T);
    return ensure_ws(p, w.total, nullptr);
}

size_t lp_saved_bytes(const lp_plan *p, int64_t B, int64_t T) {
    if (!p || B < 1 || T < 1) return 0;
    const int64_t nch = uniform_nchunks(B, T, p->L);
    return bytes_state(p->M, nch) + bytes_phi(p->M, nch);
}

size_t lp_saved_bytes_varlen(const lp_plan *p, int64_t B, int64_t N) {
    if (!p || B < 1 || N < 1) return 0;
    const int64_t nch = ceil_div(N, p->L) + B;
    return bytes_state(p->M, nch) + bytes_phi(p->M, nch);
}

int lp_forward(lp_plan *p, int64_t B, int64_t T, const float *e, const float *a, const double *zi, float *s,
               double *zf, void *saved, uint32_t *nonfinite, void *stream) {
    return forward_impl(p, B, nullptr, T, e, a, zi, s, zf, saved, stream, nullptr, nullptr, 0, false, false,
                        nonfinite);
}

int lp_forward_noalloc(lp_plan *p, int64_t B, int64_t T, const float *e, const float *a, const double *zi, float *s,
                       double *zf, void *saved, uint32_t *nonfinite, void *stream) {
    return forward_impl(p, B, nullptr, T, e, a, zi, s, zf, saved, stream, nullptr, nullptr, 0, false, true,
                        nonfinite);
}

int lp_backward(lp_plan *p, int64_t B, int64_t T, const float *g, const float *a, const float *e, const double *zi,
                const float *s, const void *saved, float *grad_e, float *grad_a, double *grad_zi,
                uint32_t *nonfinite, void *stream) {
    return backward_impl(p, B, nullptr, T, g, a, e, zi, s, saved, grad_e, grad_a, grad_zi, stream, 0, false,
                         nonfinite);
}

int lp_forward_ti(lp_plan *p, int64_t B, int64_t T, const float *e, const float *a, const double *zi, float *s,
                  double *zf, void *saved, void *stream) {
    return forward_impl(p, B, nullptr, T, e, a, zi, s, zf, saved, stream, nullptr, nullptr, 0, true);
}

int lp_backward_ti(lp_plan *p, int64_t B, int64_t T, const float *g, const float *a, const float *e,
                   const double *zi, const float *s, const void *saved, float *grad_e, float *grad_a,
                   double *grad_zi, void *stream) {
    return backward_impl(p, B, nullptr, T, g, a, e, zi, s, saved, grad_e, grad_a, grad_zi, stream, 0, true);
}

// ---- frame-rate coefficients: rows once per hop samples, interpolated in the kernels

int64_t lp_coef_frames_count(int64_t T, int64_t hop) { return (T < 1 || hop < 1) ? 0 : (T - 1) / hop + 2; }

}  // extern "C"

namespace {

// Validates a frame-rate call and fills the frame fields of the sequence view.
template <class O>
int frames_setup(const lp_plan *p, int64_t T, int64_t hop, typename O::Bufs &w) {
    const int nf = (int)((p->L - 1) / hop + 3);
    if (!O::frames_lds_ok(p->L, nf))
        return fail(LP_EINVAL, "hop %lld is too short for chunk length %d: the staged frame rows do not fit in LDS",
                    (long long)hop, p->L);
    w.S.hop = (int)hop;
    w.S.nf = nf;
    w.S.F = lp_coef_frames_count(T, hop);
    return LP_OK;
}

int frames_args(int64_t B, int64_t T, int64_t hop) {
    if (B < 1) return fail(LP_EINVAL, "B must be >= 1 (got %lld)", (long long)B);
    if (T < 1) return fail(LP_EINVAL, "T must be >= 1 (got %lld)", (long long)T);
    if (hop < 1 || hop > (1 << 20)) return fail(LP_EINVAL, "hop must be in [1, 2^20] (got %lld)", (long long)hop);
    return LP_OK;
}

}  // namespace

extern "C" {

int lp_forward_frames(lp_plan *p, int64_t B, int64_t T, int64_t hop, const float *e, const float *A,
                      const double *zi, float *s, double *zf, void *saved, void *stream) {
    if (int r = check_plan(p)) return r;
    if (int r = frames_args(B, T, hop)) return r;
    if (!e || !A || !s) return fail(LP_EINVAL, "e, A and s are required");
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(LP_EDEVICE, "cannot select device %d", p->device);
    hipStream_t st = (hipStream_t)stream;
    int rc = LP_OK;
    Timer tm{p, st};
    dispatch(p->M, [&](auto ops) {
        using O = decltype(ops);
        typename O::Bufs w;
        rc = prepare<O>(p, B, nullptr, T, saved, st, w);
        if (rc == LP_OK) rc = frames_setup<O>(p, T, hop, w);
        if (rc == LP_OK) O::template forward_t<true>(w, e, A, zi, s, zf, st, tm);
    });
    if (rc != LP_OK) return rc;
    return check_hip(hipGetLastError(), "kernel launch (frame-rate forward)");
}

int lp_backward_frames(lp_plan *p, int64_t B, int64_t T, int64_t hop, const float *g, const float *A,
                       const float *e, const double *zi, const float *s, const void *saved, float *grad_e,
                       float *grad_A, double *grad_zi, void *stream) {
    if (int r = check_plan(p)) return r;
    if (int r = frames_args(B, T, hop)) return r;
    if (!g || !A || !saved) return fail(LP_EINVAL, "g, A and saved are required");
    if ((grad_e || grad_A) && !s && !e) return fail(LP_EINVAL, "the adjoint needs s or e (to recompute s)");
    if (!grad_e && !grad_A && !grad_zi) return LP_OK;
    (void)zi;
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(LP_EDEVICE, "cannot select device %d", p->device);
    hipStream_t st = (hipStream_t)stream;
    int rc = LP_OK;
    Timer tm{p, st};
    dispatch(p->M, [&](auto ops) {
        using O = decltype(ops);
        typename O::Bufs w;
        const int64_t nch = B * ceil_div(T, p->L);
        const int nf = (int)((p->L - 1) / hop + 3);
        rc = prepare<O>(p, B, nullptr, T, saved, st, w, nullptr, nullptr, 0,
                        grad_A ? (size_t)nch * nf * p->M * sizeof(double) : 0);
        if (rc == LP_OK) rc = frames_setup<O>(p, T, hop, w);
        if (rc == LP_OK) O::template backward_t<true>(w, g, A, e, s, grad_e, grad_A, grad_zi, st, tm);
    });
    if (rc != LP_OK) return rc;
    return check_hip(hipGetLastError(), "kernel launch (frame-rate backward)");
}

int64_t lp_frames_count(int64_t T, int64_t hop) { return (T < 1 || hop < 1) ? 0 : ceil_div(T, hop) + 3; }

static int frames_launch(bool gather, int64_t B, int64_t T, int64_t hop, const float *src, float *dst, int weighted,
                         void *stream) {
    if (B < 1 || T < 1 || hop < 1) return fail(LP_EINVAL, "B, T and hop must be >= 1");
    if (!src || !dst) return fail(LP_EINVAL, "input and output are required");
    const int64_t F = ceil_div(T, hop) + 3, n = gather ? B * F * 4 * hop : B * T;
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(n, 256), 65536);
    if (gather)
        hipLaunchKernelGGL(k_frames_gather, dim3(grid), dim3(256), 0, (hipStream_t)stream, B, T, hop, F, src, dst,
                           weighted);
    else
        hipLaunchKernelGGL(k_frames_overlap_add, dim3(grid), dim3(256), 0, (hipStream_t)stream, B, T, hop, F, src,
                           dst, weighted);
    return check_hip(hipGetLastError(), gather ? "kernel launch (frames gather)" : "kernel launch (overlap-add)");
}

int lp_frames_gather(int64_t B, int64_t T, int64_t hop, const float *x, float *xf, int weighted, void *stream) {
    return frames_launch(true, B, T, hop, x, xf, weighted, stream);
}

int lp_frames_overlap_add(int64_t B, int64_t T, int64_t hop, const float *xf, float *x, int weighted, void *stream) {
    return frames_launch(false, B, T, hop, xf, x, weighted, stream);
}

int lp_plan_autotune(lp_plan *p, int64_t B, int64_t T, int reps, int *chosen, double *best_ms) {
    if (int r = check_plan(p)) return r;
    if (B < 1 || T < 1) return fail(LP_EINVAL, "B and T must be >= 1");
    if (reps < 1) reps = 3;
    if (p->live_graphs > 0)
        return fail(LP_EINVAL, "cannot autotune while %d captured graph(s) use the plan", p->live_graphs);
    const int M = p->M;
    // the timed batch keeps T and at most ~32 M samples (beyond that every candidate fills the chip)
    const int64_t Bt = std::max<int64_t>(1, std::min<int64_t>(B, (int64_t(1) << 25) / T));
    DeviceGuard dg(p->device);
    int maxL = 0;
    dispatch(M, [&](auto ops) { maxL = decltype(ops)::max_chunk(); });
    // candidates about 6 % apart from 64 to 1024 samples, as multiples of M: step
    // time is not smooth in L (the chunk stride meets the memory interleave
    // differently at neighbouring lengths), so the grid is dense
    std::vector<int> cands;
    if (p->flags & LP_FLAG_HIGH_RADIUS) {
        // high-radius plans: only chunk lengths long enough for the chained carry's accuracy
        const int lo = std::min(kAccurateChunk, maxL);
        for (double target = lo; target <= maxL * 1.001; target *= 1.06) {
            const int L = std::min(maxL, std::max(1, (int(target) + M - 1) / M) * M);
            if (std::find(cands.begin(), cands.end(), L) == cands.end()) cands.push_back(L);
        }
        if (std::find(cands.begin(), cands.end(), maxL) == cands.end()) cands.push_back(maxL);
    } else {
        for (double target = 64.0; target <= 1024.0 * 1.001; target *= 1.06) {
            const int L = std::max(1, (int(target) + M / 2) / M) * M;
            if (L <= maxL && std::find(cands.begin(), cands.end(), L) == cands.end()) cands.push_back(L);
        }
    }
    const int oldL = p->L;
    size_t saved_bytes = 0;  // the smallest chunk length needs the most saved state
    for (int L : cands) {
        p->L = L;
        saved_bytes = std::max(saved_bytes, lp_saved_bytes(p, Bt, T));
    }
    p->L = oldL;
    const size_t n = (size_t)Bt * T;
    float *buf = nullptr;
    const size_t floats = n * (size_t)(2 * M + 4);  // e, g, s, ge, a, ga
    const size_t bytes = floats * sizeof(float) + saved_bytes;
    if (hipMalloc(&buf, bytes) != hipSuccess) return fail(LP_ENOMEM, "autotune buffers (%zu bytes)", bytes);
    int rc = check_hip(hipMemset(buf, 0, floats * sizeof(float)), "autotune memset");
    float *e = buf, *g = e + n, *s = g + n, *ge = s + n, *a = ge + n, *ga = a + n * M;
    void *saved = ga + n * M;
    // e and g uniform in [-1, 1); coefficients below 0.9 / M in magnitude (a stable
    // filter: their absolute sum stays below 0.9)
    if (rc == LP_OK) {
        hipLaunchKernelGGL(k_tune_fill, dim3(1024), dim3(256), 0, nullptr, e, (int64_t)(2 * n), 1.0f, 1u);
        hipLaunchKernelGGL(k_tune_fill, dim3(1024), dim3(256), 0, nullptr, a, (int64_t)(n * M), 0.9f / M, 2u);
        rc = check_hip(hipStreamSynchronize(nullptr), "autotune input fill");
    }
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == LP_OK && (hipStreamCreate(&st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
                        hipEventCreate(&e1) != hipSuccess))
        rc = fail(LP_EDEVICE, "autotune stream/event creation failed");
    const bool timing = p->timing;
    p->timing = false;
    // carry modes: both unless the caller fixed one
    const int oldflags = p->flags;
    const int chained_now = (p->flags & LP_FLAG_CHAINED_CARRY) ? 1 : 0;
    const int modes[2] = {p->carry_fixed ? chained_now : 0, 1};
    const int nmodes = p->carry_fixed ? 1 : 2;
    int bestL = oldL, best_mode = chained_now;
    float best = 1e30f;
    for (int mi = 0; mi < nmodes * (int)cands.size(); ++mi) {
        if (rc != LP_OK) break;
        const int L = cands[mi % cands.size()], mode = modes[mi / cands.size()];
        p->L = L;
        p->flags = mode ? (oldflags | LP_FLAG_CHAINED_CARRY) : (oldflags & ~LP_FLAG_CHAINED_CARRY);
        float bestL_ms = 1e30f;
        for (int r = 0; r <= reps && rc == LP_OK; ++r) {  // r = 0 warms up (and sizes the workspace)
            (void)hipEventRecord(e0, st);
            rc = lp_forward(p, Bt, T, e, a, nullptr, s, nullptr, saved, nullptr, st);
            if (rc == LP_OK) rc = lp_backward(p, Bt, T, g, a, e, nullptr, nullptr, saved, ge, ga, nullptr, nullptr, st);
            (void)hipEventRecord(e1, st);
            if (rc == LP_OK) rc = check_hip(hipEventSynchronize(e1), "autotune sync");
            float ms = 0.f;
            if (rc == LP_OK && r > 0 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) bestL_ms = std::min(bestL_ms, ms);
        }
        if (rc == LP_OK && bestL_ms < best) {
            best = bestL_ms;
            bestL = L;
            best_mode = mode;
        }
    }
    p->timing = timing;
    p->L = rc == LP_OK ? bestL : oldL;
    p->flags = rc == LP_OK ? (best_mode ? (oldflags | LP_FLAG_CHAINED_CARRY) : (oldflags & ~LP_FLAG_CHAINED_CARRY))
                           : oldflags;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(buf);
    if (rc == LP_OK) rc = lp_plan_status(p);  // a scan timeout during tuning is an error, not a choice
    if (rc != LP_OK) return rc;
    if (chosen) *chosen = bestL;
    if (best_ms) *best_ms = (double)best;
    return LP_OK;
}

int lp_forward_varlen(lp_plan *p, int64_t B, const int64_t *offsets, int64_t N, const float *e, const float *a,
                      const double *zi, float *s, double *zf, void *saved, void *stream) {
    if (!offsets) return fail(LP_EINVAL, "offsets is NULL");
    return forward_impl(p, B, offsets, N, e, a, zi, s, zf, saved, stream);
}

int lp_backward_varlen(lp_plan *p, int64_t B, const int64_t *offsets, int64_t N, const float *g, const float *a,
                       const float *e, const double *zi, const float *s, const void *saved, float *grad_e,
                       float *grad_a, double *grad_zi, void *stream) {
    if (!offsets) return fail(LP_EINVAL, "offsets is NULL");
    return backward_impl(p, B, offsets, N, g, a, e, zi, s, saved, grad_e, grad_a, grad_zi, stream);
}

int lp_forward_segments(lp_plan *p, int64_t B, const int64_t *starts, const int64_t *lens, int64_t N,
                        int64_t total_bound, const float *e, const float *a, const double *zi, float *s, double *zf,
                        void *stream) {
    if (!starts || !lens) return fail(LP_EINVAL, "starts and lens are required");
    if (total_bound < 0) return fail(LP_EINVAL, "total_bound must be >= 0");
    return forward_impl(p, B, nullptr, N, e, a, zi, s, zf, nullptr, stream, starts, lens, total_bound);
}

int lp_forward_plain(int M, int64_t B, int64_t T, const float *e, const float *a, const double *zi, float *s,
                     double *zf, void *stream) {
    if (M < 1 || M > 64) return fail(LP_EINVAL, "order M must be in [1, 64] (got %d)", M);
    if (B < 1 || T < 1) return fail(LP_EINVAL, "B and T must be >= 1");
    if (!e || !a || !s) return fail(LP_EINVAL, "e, a and s are required");
    const bool ok = dispatch(M, [&](auto ops) { decltype(ops)::plain_fwd(B, T, e, a, zi, s, zf, (hipStream_t)stream); });
    if (!ok) return fail(LP_EINVAL, "order M = %d is not compiled", M);
    return check_hip(hipGetLastError(), "kernel launch (plain forward)");
}

int lp_backward_plain(int M, int64_t B, int64_t T, const float *g, const float *a, const double *zi, const float *s,
                      float *grad_e, float *grad_a, double *grad_zi, void *stream) {
    if (M < 1 || M > 64) return fail(LP_EINVAL, "order M must be in [1, 64] (got %d)", M);
    if (B < 1 || T < 1) return fail(LP_EINVAL, "B and T must be >= 1");
    if (!g || !a) return fail(LP_EINVAL, "g and a are required");
    if (grad_a && !s) return fail(LP_EINVAL, "grad_a needs the forward output s");
    const bool ok = dispatch(M, [&](auto ops) {
        decltype(ops)::plain_bwd(B, T, g, a, zi, s, grad_e, grad_a, grad_zi, (hipStream_t)stream);
    });
    if (!ok) return fail(LP_EINVAL, "order M = %d is not compiled", M);
    return check_hip(hipGetLastError(), "kernel launch (plain backward)");
}

size_t lp_saved_bytes_pair(const lp_plan *p, int64_t B, int64_t T) { return lp_saved_bytes(p, 2 * B, T); }

int lp_forward_pair(lp_plan *p, int64_t B, int64_t T, const float *e2, const float *a2, float *y, float *s2,
                    void *saved, void *stream) {
    if (!y || !s2) return fail(LP_EINVAL, "y and s2 are required");
    if (B < 1 || T < 1) return fail(LP_EINVAL, "B and T must be >= 1");
    if (int r = forward_impl(p, 2 * B, nullptr, T, e2, a2, nullptr, s2, nullptr, saved, stream)) return r;
    DeviceGuard dg(p->device);
    const int64_t n = B * T;
    const unsigned grid = (unsigned)ceil_div(ceil_div(n, 4), 256);
    Timer tm{p, (hipStream_t)stream};
    tm.begin("pair_sum");
    const int vec = ((uintptr_t)y % 16 == 0) && ((uintptr_t)s2 % 16 == 0) && (n % 4 == 0);
    hipLaunchKernelGGL(k_pair_sum, dim3(grid), dim3(256), 0, (hipStream_t)stream, y, s2, n, vec);
    tm.end();
    return check_hip(hipGetLastError(), "kernel launch (pair sum)");
}

int lp_backward_pair(lp_plan *p, int64_t B, int64_t T, const float *g, const float *a2, const float *e2,
                     const float *s2, const void *saved, float *ge2, float *ga2, void *stream) {
    if (B < 1 || T < 1) return fail(LP_EINVAL, "B and T must be >= 1");
    return backward_impl(p, 2 * B, nullptr, T, g, a2, e2, nullptr, s2, saved, ge2, ga2, nullptr, stream, B);
}

}  // extern "C"

struct lp_graph {
    int device;
    hipGraph_t graph;
    hipGraphExec_t exec;
    lp_plan *plan;  // whose workspace the graph's kernels address
};

extern "C" {

int lp_graph_capture_pair_step(lp_plan *p, int64_t B, int64_t T, const float *e2, const float *a2, float *y,
                               float *s2, void *saved, const float *g, float *ge2, float *ga2, int store_s,
                               lp_graph **out) {
    if (!out) return fail(LP_EINVAL, "out is NULL");
    *out = nullptr;
    if (int r = check_plan(p)) return r;
    if (int r = lp_plan_reserve(p, 2 * B, T)) return r;
    DeviceGuard dg(p->device);
    const bool timing = p->timing;
    p->timing = false;
    hipStream_t st = nullptr;
    if (hipStreamCreate(&st) != hipSuccess) {
        p->timing = timing;
        return fail(LP_EDEVICE, "stream creation failed");
    }
    int rc = LP_OK;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = fail(LP_EDEVICE, "hipStreamBeginCapture failed");
    } else {
        rc = lp_forward_pair(p, B, T, e2, a2, y, s2, saved, st);
        if (rc == LP_OK) rc = lp_backward_pair(p, B, T, g, a2, e2, store_s ? s2 : nullptr, saved, ge2, ga2, st);
        const hipError_t ec = hipStreamEndCapture(st, &graph);
        if (rc == LP_OK && ec != hipSuccess) rc = fail(LP_EDEVICE, "hipStreamEndCapture failed");
    }
    p->timing = timing;
    lp_graph *gr = nullptr;
    if (rc == LP_OK) {
        gr = new (std::nothrow) lp_graph{p->device, graph, nullptr, p};
        if (!gr) rc = fail(LP_ENOMEM, "out of host memory");
    }
    if (rc == LP_OK && hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0) != hipSuccess)
        rc = fail(LP_EDEVICE, "hipGraphInstantiate failed");
    (void)hipStreamDestroy(st);
    if (rc != LP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        delete gr;
        return rc;
    }
    ++p->live_graphs;
    *out = gr;
    return LP_OK;
}

int lp_graph_launch(lp_graph *gr, void *stream) {
    if (!gr) return fail(LP_EINVAL, "graph is NULL");
    DeviceGuard dg(gr->device);
    return check_hip(hipGraphLaunch(gr->exec, (hipStream_t)stream), "hipGraphLaunch");
}

int lp_graph_destroy(lp_graph *gr) {
    if (!gr) return LP_OK;
    DeviceGuard dg(gr->device);
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    if (gr->plan && gr->plan->live_graphs > 0) --gr->plan->live_graphs;
    delete gr;
    return LP_OK;
}

}  // extern "C"
