// Wilson hopping stencil for the dense SU(N > 2) link formats (CPLX3, CPLX4,
// CPLX6, CPLX10, REAL8, REAL15, SU3_ROW2): the same kernel template as the
// SU(2) formats with N x N colour products; clover epilogues for the SU(3)
// fundamental formats.
#include "hop_lanes.h"
#include "hop_quad.h"

// REAL8 links in FP64 run on the four-lanes-per-site kernel of hop_quad.h,
// CPLX10 links in FP64 on that of hop_lanes.h
namespace hrd {

namespace {

template <typename S>
hipError_t dense_hop_for(int rep, const HopArgs &a, bool dag, bool has_a, bool norm, bool full, hipStream_t st,
                         int clov)
{
    if constexpr (std::is_same<S, double>::value) {
        if (quad_covers(rep, full, a.g.Vh)) return launch_hop_quad(a, dag, has_a, norm, st);
        if (lanes_covers(rep, full, a.g.Vh)) return launch_hop_lanes<HRD_CPLX10>(a, dag, has_a, norm, st);
    }
    switch (rep) {
        case HRD_CPLX3: return dispatch_hop_clov<HRD_CPLX3, S>(a, dag, has_a, norm, full, st, clov);
        case HRD_CPLX4: return dispatch_hop<HRD_CPLX4, S, CLOV_NONE>(a, dag, has_a, norm, full, st);
        case HRD_CPLX6: return dispatch_hop<HRD_CPLX6, S, CLOV_NONE>(a, dag, has_a, norm, full, st);
        case HRD_CPLX10: return dispatch_hop<HRD_CPLX10, S, CLOV_NONE>(a, dag, has_a, norm, full, st);
        case HRD_REAL15: return dispatch_hop<HRD_REAL15, S, CLOV_NONE>(a, dag, has_a, norm, full, st);
        case HRD_SU3_ROW2: return dispatch_hop_clov<HRD_SU3_ROW2, S>(a, dag, has_a, norm, full, st, clov);
        default: return dispatch_hop<HRD_REAL8, S, CLOV_NONE>(a, dag, has_a, norm, full, st);
    }
}

template <typename S>
hipError_t dense_rupd_for(int rep, const HopArgs &a, hipStream_t st, int clov)
{
    if constexpr (std::is_same<S, double>::value) {
        if (quad_covers(rep, false, a.g.Vh)) return launch_hop_quad_rupdate(a, st);
        if (lanes_covers(rep, false, a.g.Vh)) return launch_hop_lanes_rupdate<HRD_CPLX10>(a, st);
    }
    switch (rep) {
        case HRD_CPLX3: return dispatch_rupd<HRD_CPLX3, S>(a, st, clov);
        case HRD_CPLX4: return dispatch_rupd<HRD_CPLX4, S>(a, st, CLOV_NONE);
        case HRD_CPLX6: return dispatch_rupd<HRD_CPLX6, S>(a, st, CLOV_NONE);
        case HRD_CPLX10: return dispatch_rupd<HRD_CPLX10, S>(a, st, CLOV_NONE);
        case HRD_REAL15: return dispatch_rupd<HRD_REAL15, S>(a, st, CLOV_NONE);
        case HRD_SU3_ROW2: return dispatch_rupd<HRD_SU3_ROW2, S>(a, st, clov);
        default: return dispatch_rupd<HRD_REAL8, S>(a, st, CLOV_NONE);
    }
}

}  // namespace

hipError_t launch_hop_dense(int rep, int prec, const HopArgs &a, bool dag, bool has_a, bool norm, bool full,
                            hipStream_t st, int clov)
{
    switch (prec) {
        case HRD_F64: return dense_hop_for<double>(rep, a, dag, has_a, norm, full, st, clov);
        case HRD_F32: return dense_hop_for<float>(rep, a, dag, has_a, norm, full, st, clov);
        default: return dense_hop_for<h16>(rep, a, dag, has_a, norm, full, st, clov);
    }
}

hipError_t launch_hop_rupdate_dense(int rep, int prec, const HopArgs &a, hipStream_t st, int clov)
{
    switch (prec) {
        case HRD_F64: return dense_rupd_for<double>(rep, a, st, clov);
        case HRD_F32: return dense_rupd_for<float>(rep, a, st, clov);
        default: return dense_rupd_for<h16>(rep, a, st, clov);
    }
}

}  // namespace hrd
