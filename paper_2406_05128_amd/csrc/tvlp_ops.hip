// Instantiates the launch sequences of one filter order (TVLP_ORDER, set by the
// build), or of every compiled order when it is not set.
#include "tvlp_ops_impl.hpp"

#define TVLP_INSTANTIATE(m)                                                                                     \
    template struct tvlp_host::Ops<m>;                                                                          \
    template void tvlp_host::Ops<m>::forward_t<false>(const tvlp_host::Ops<m>::Bufs &, const float *,         \
                                                       const float *, const double *, float *, double *,       \
                                                       hipStream_t, tvlp_host::Timer &);                       \
    template void tvlp_host::Ops<m>::forward_t<true>(const tvlp_host::Ops<m>::Bufs &, const float *,          \
                                                      const float *, const double *, float *, double *,        \
                                                      hipStream_t, tvlp_host::Timer &);                        \
    template void tvlp_host::Ops<m>::backward_t<false>(const tvlp_host::Ops<m>::Bufs &, const float *,        \
                                                        const float *, const float *, const float *, float *,  \
                                                        float *, double *, hipStream_t, tvlp_host::Timer &);   \
    template void tvlp_host::Ops<m>::backward_t<true>(const tvlp_host::Ops<m>::Bufs &, const float *,         \
                                                       const float *, const float *, const float *, float *,   \
                                                       float *, double *, hipStream_t, tvlp_host::Timer &);

#ifdef TVLP_ORDER
TVLP_INSTANTIATE(TVLP_ORDER)
#else
TVLP_INSTANTIATE(1)
TVLP_INSTANTIATE(2)
TVLP_INSTANTIATE(3)
TVLP_INSTANTIATE(4)
TVLP_INSTANTIATE(6)
TVLP_INSTANTIATE(8)
TVLP_INSTANTIATE(10)
TVLP_INSTANTIATE(12)
TVLP_INSTANTIATE(16)
TVLP_INSTANTIATE(20)
TVLP_INSTANTIATE(22)
TVLP_INSTANTIATE(24)
TVLP_INSTANTIATE(32)
#endif
