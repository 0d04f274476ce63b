// Host side of the C ABI declared in include/tvlp.h: plans, argument checks,
// workspace management and kernel dispatch over the compiled filter orders.
#include "tvlp.h"
#include "tvlp_device.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

using namespace tvlp;

struct TimingRecord {
    const char *name;
    hipEvent_t start, stop;
};

struct lp_plan {
    int device;
    int M;
    int L;
    int flags;
    void *ws;
    size_t ws_bytes;
    bool timing;
    std::vector<TimingRecord> pending;
    std::map<std::string, std::pair<double, int64_t>> totals;  // name -> (ms, launches)
};

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

int check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return LP_OK;
    return fail(LP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

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

int default_chunk(int M) {
    int mult = (256 + M - 1) / M;
    return std::max(1, mult) * M;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

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

// Workspace layout for one call with nch chunks and n samples over B sequences.
struct WsLayout {
    size_t xs, phi, z, q, yend, sbuf, cbase, total;
};

WsLayout ws_layout(int M, int64_t nch, int64_t nsamp, int64_t B) {
    WsLayout w{};
    size_t off = 0;
    w.xs = off;   off += align_up(bytes_state(M, nch));
    w.phi = off;  off += align_up(bytes_phi(M, nch));
    w.z = off;    off += align_up(bytes_state(M, nch));
    w.q = off;    off += align_up(bytes_state(M, nch));
    w.yend = off; off += align_up(bytes_state(M, nch));
    w.sbuf = off; off += align_up((size_t)nsamp * sizeof(float));
    w.cbase = off; off += align_up((size_t)(B + 1) * sizeof(int64_t));
    w.total = off;
    return w;
}

int ensure_ws(lp_plan *p, size_t need, hipStream_t stream) {
    if (p->ws_bytes >= need) return LP_OK;
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
    p->ws = ptr;
    p->ws_bytes = need;
    return LP_OK;
}

// Prefix of chunk counts over a packed varlen batch (single block).
__global__ __launch_bounds__(1024) void k_build_cbase(const int64_t *__restrict__ offsets, int64_t n, int L,
                                                      int64_t N, int64_t *__restrict__ cbase) {
    __shared__ int64_t part[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += 1024) {
        const int64_t b = base + threadIdx.x;
        int64_t cnt = 0;
        if (b < n) {
            // same clamping as seq_view
            const int64_t lo = min(max(offsets[b], (int64_t)0), N);
            const int64_t hi = min(max(offsets[b + 1], lo), N);
            const int64_t len = hi - lo;
            cnt = len <= 0 ? 0 : (len + L - 1) / L;
        }
        part[threadIdx.x] = cnt;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            int64_t v = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0;
            __syncthreads();
            part[threadIdx.x] += v;
            __syncthreads();
        }
        if (b < n) cbase[b + 1] = carry + part[threadIdx.x];
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) cbase[0] = 0;
}

template <int M>
struct Ops {
    using BS = BasisShape<M>;
    static constexpr int CPW = 64 / BS::LPC;

    static void forward(const Seqs &S, int64_t nch, int64_t nseq, const float *e, const float *a,
                        const double *zi, float *s, double *zf, double *xs, double *phi, double *z,
                        hipStream_t st, Timer &tm) {
        if (nch <= 0) return;
        tm.begin("fwd_basis");
        hipLaunchKernelGGL((k_fwd_basis<M, BS::LPC, BS::CPL>), dim3((unsigned)ceil_div(nch, CPW)), dim3(64), 0, st,
                           S, e, a, phi, z, nch);
        tm.end();
        tm.begin("fwd_chain");
        hipLaunchKernelGGL((k_fwd_chain<M>), dim3((unsigned)nseq), dim3(64), 0, st, S, phi, z, zi, xs);
        tm.end();
        tm.begin("fwd_emit");
        hipLaunchKernelGGL((k_fwd_emit<M>), dim3((unsigned)ceil_div(nch, 64)), dim3(64), 0, st, S, e, a, xs, s,
                           zf, nch);
        tm.end();
    }

    static void backward(const Seqs &S, int64_t nch, int64_t nseq, const float *g, const float *a,
                         const float *e, const float *s_in, const double *xs, const double *phi, double *q,
                         double *yend, float *sbuf, float *ge, float *ga, double *gzi, hipStream_t st,
                         Timer &tm) {
        if (nch <= 0) return;
        tm.begin("bwd_zs");
        hipLaunchKernelGGL((k_bwd_zs<M>), dim3((unsigned)ceil_div(nch, 64)), dim3(64), 0, st, S, g, a, q, nch,
                           gzi ? 1 : 0);
        tm.end();
        tm.begin("bwd_chain");
        hipLaunchKernelGGL((k_bwd_chain<M>), dim3((unsigned)nseq), dim3(64), 0, st, S, phi, q, yend, gzi);
        tm.end();
        const float *s = s_in;
        if (ga && !s) {
            tm.begin("recompute_s");
            hipLaunchKernelGGL((k_recompute_s<M>), dim3((unsigned)ceil_div(nch, 64)), dim3(64), 0, st, S, e, a,
                               xs, sbuf, nch);
            tm.end();
            s = sbuf;
        }
        tm.begin("bwd_emit");
        if (ga)
            hipLaunchKernelGGL((k_bwd_emit<M, true>), dim3((unsigned)ceil_div(nch, 64)), dim3(64), 0, st, S, g,
                               a, s, xs, yend, ge, ga, nch);
        else if (ge)
            hipLaunchKernelGGL((k_bwd_emit<M, false>), dim3((unsigned)ceil_div(nch, 64)), dim3(64), 0, st, S, g,
                               a, s, xs, yend, ge, ga, nch);
        tm.end();
    }

    static void plain_fwd(int64_t B, int64_t T, const float *e, const float *a, const double *zi, float *s,
                          double *zf, hipStream_t st) {
        hipLaunchKernelGGL((k_plain_fwd<M>), dim3((unsigned)ceil_div(B, 64)), dim3(64), 0, st, B, T, e, a, zi, s,
                           zf);
    }

    static void plain_bwd(int64_t B, int64_t T, const float *g, const float *a, const double *zi, const float *s,
                          float *ge, float *ga, double *gzi, hipStream_t st) {
        if (ga)
            hipLaunchKernelGGL((k_plain_bwd<M, true>), dim3((unsigned)ceil_div(B, 64)), dim3(64), 0, st, B, T, g,
                               a, zi, s, ge, ga, gzi);
        else
            hipLaunchKernelGGL((k_plain_bwd<M, false>), dim3((unsigned)ceil_div(B, 64)), dim3(64), 0, st, B, T, g,
                               a, zi, s, ge, ga, gzi);
    }
};

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

// Common driver of the uniform and varlen forward.
int forward_impl(lp_plan *p, int64_t B, const int64_t *offsets, int64_t T_or_N, const float *e, const float *a,
                 const double *zi, float *s, double *zf, void *saved, void *stream) {
    if (int r = check_plan(p)) return r;
    if (B < 1) return fail(LP_EINVAL, "B must be >= 1 (got %lld)", (long long)B);
    if (T_or_N < 1) return fail(LP_EINVAL, "T (or N) must be >= 1 (got %lld)", (long long)T_or_N);
    if (!e || !a || !s) return fail(LP_EINVAL, "e, a and s are required");
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(LP_EDEVICE, "cannot select device %d", p->device);
    hipStream_t st = (hipStream_t)stream;
    const int M = p->M, L = p->L;
    const int64_t nsamp = offsets ? T_or_N : B * T_or_N;
    const int64_t nch = offsets ? ceil_div(T_or_N, L) + B : uniform_nchunks(B, T_or_N, L);
    WsLayout w = ws_layout(M, nch, 0, B);
    if (int r = ensure_ws(p, w.total, st)) return r;
    char *ws = (char *)p->ws;
    double *xs = saved ? (double *)saved : (double *)(ws + w.xs);
    double *phi = saved ? (double *)((char *)saved + bytes_state(M, nch)) : (double *)(ws + w.phi);
    Seqs S{nullptr, nullptr, offsets ? 0 : T_or_N, B, L, offsets ? T_or_N : 0, nch};
    if (offsets) {
        int64_t *cb = (int64_t *)(ws + w.cbase);
        hipLaunchKernelGGL(k_build_cbase, dim3(1), dim3(1024), 0, st, offsets, B, L, T_or_N, cb);
        S.offsets = offsets;
        S.cbase = cb;
    }
    (void)nsamp;
    Timer tm{p, st};
    dispatch(M, [&](auto ops) {
        decltype(ops)::forward(S, nch, B, e, a, zi, s, zf, xs, phi, (double *)(ws + w.z), st, tm);
    });
    return check_hip(hipGetLastError(), "kernel launch (forward)");
}

int backward_impl(lp_plan *p, int64_t B, const int64_t *offsets, int64_t T_or_N, const float *g, const float *a,
                  const float *e, const double *zi, const float *s, const void *saved, float *ge, float *ga,
                  double *gzi, void *stream) {
    if (int r = check_plan(p)) return r;
    if (B < 1) return fail(LP_EINVAL, "B must be >= 1 (got %lld)", (long long)B);
    if (T_or_N < 1) return fail(LP_EINVAL, "T (or N) must be >= 1 (got %lld)", (long long)T_or_N);
    if (!g || !a || !saved) return fail(LP_EINVAL, "g, a and saved are required");
    if (ga && !s && !e) return fail(LP_EINVAL, "grad_a needs s or e (to recompute s)");
    if (!ge && !ga && !gzi) return LP_OK;
    (void)zi;
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(LP_EDEVICE, "cannot select device %d", p->device);
    hipStream_t st = (hipStream_t)stream;
    const int M = p->M, L = p->L;
    const int64_t nsamp = offsets ? T_or_N : B * T_or_N;
    const int64_t nch = offsets ? ceil_div(T_or_N, L) + B : uniform_nchunks(B, T_or_N, L);
    WsLayout w = ws_layout(M, nch, (ga && !s) ? nsamp : 0, B);
    if (int r = ensure_ws(p, w.total, st)) return r;
    char *ws = (char *)p->ws;
    const double *xs = (const double *)saved;
    const double *phi = (const double *)((const char *)saved + bytes_state(M, nch));
    Seqs S{nullptr, nullptr, offsets ? 0 : T_or_N, B, L, offsets ? T_or_N : 0, nch};
    if (offsets) {
        int64_t *cb = (int64_t *)(ws + w.cbase);
        hipLaunchKernelGGL(k_build_cbase, dim3(1), dim3(1024), 0, st, offsets, B, L, T_or_N, cb);
        S.offsets = offsets;
        S.cbase = cb;
    }
    Timer tm{p, st};
    dispatch(M, [&](auto ops) {
        decltype(ops)::backward(S, nch, B, g, a, e, s, xs, phi, (double *)(ws + w.q), (double *)(ws + w.yend),
                                (float *)(ws + w.sbuf), ge, ga, gzi, st, tm);
    });
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
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(LP_EINVAL, "device %d not available", device);
    lp_plan *p = new (std::nothrow) lp_plan{};
    if (!p) return fail(LP_ENOMEM, "out of host memory");
    p->device = device;
    p->M = M;
    p->L = default_chunk(M);
    p->flags = flags;
    *out = p;
    return LP_OK;
}

int lp_plan_destroy(lp_plan *p) {
    if (!p) return LP_OK;
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
    p->L = L;
    return LP_OK;
}

int lp_plan_get_chunk(const lp_plan *p) { return p ? p->L : 0; }

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
    WsLayout w = ws_layout(p->M, nch, B * T, B);
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
               double *zf, void *saved, void *stream) {
    return forward_impl(p, B, nullptr, T, e, a, zi, s, zf, saved, stream);
}

int lp_backward(lp_plan *p, int64_t B, int64_t T, const float *g, const float *a, const float *e, const double *zi,
                const float *s, const void *saved, float *grad_e, float *grad_a, double *grad_zi, void *stream) {
    return backward_impl(p, B, nullptr, T, g, a, e, zi, s, saved, grad_e, grad_a, grad_zi, stream);
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

}  // extern "C"
