// Wilson hopping stencil for the SU(2) link formats: slab choice, launch
// geometry and dispatch over precision, representation and epilogue (the
// kernel templates are in hop.h).
#include "hop.h"

namespace hrd {

// Widest x1-slab whose t-slice holds at most kSlabSites = 6 * 48 * 48 / 2
// sites per parity (the best of the widths measured on 48^4, where one FP64
// source slice is then 0.9 MB and the t-1, t, t+1 slices stay in a 4 MB L2).
int choose_slab(const int dims[4])
{
    constexpr long kSlabSites = 6912;
    const long R = (long)dims[2] * dims[3] / 2;
    int best = 1;
    for (int b = 1; b <= dims[1]; b++)
        if (dims[1] % b == 0 && (long)b * R <= kSlabSites) best = b;
    return best;
}

// Slab of the FULL kernel (both parities in one launch, temporal link loads):
// its t-window holds the links shared by the two parities as well, so the
// FP64 budget is half the single-parity one (measured at 48^4: FP64 plain D
// 821 -> 742 us with slab 3 instead of 6; FP32 best at the default slab).
int choose_slab_full(const int dims[4], int prec)
{
    const long budget = prec == HRD_F64 ? 3456 : 6912;
    const long R = (long)dims[2] * dims[3] / 2;
    int best = 1;
    for (int b = 1; b <= dims[1]; b++)
        if (dims[1] % b == 0 && (long)b * R <= budget) best = b;
    return best;
}

namespace {

template <typename S>
hipError_t rupd_for(int rep, const HopArgs &a, hipStream_t st, int clov)
{
    switch (rep) {
        case HRD_FUND: return dispatch_rupd<HRD_FUND, S>(a, st, clov);
        case HRD_ADJ: return dispatch_rupd<HRD_ADJ, S>(a, st, clov);
        case HRD_FUND_SU2: return dispatch_rupd<HRD_FUND_SU2, S>(a, st, clov);
        default: return dispatch_rupd<HRD_ADJ_SU2, S>(a, st, clov);
    }
}

template <typename S>
hipError_t hop_for(int rep, const HopArgs &a, bool dag, bool has_a, bool norm, bool full, hipStream_t st, int clov)
{
    switch (rep) {
        case HRD_FUND: return dispatch_hop_clov<HRD_FUND, S>(a, dag, has_a, norm, full, st, clov);
        case HRD_ADJ: return dispatch_hop_clov<HRD_ADJ, S>(a, dag, has_a, norm, full, st, clov);
        case HRD_FUND_SU2: return dispatch_hop_clov<HRD_FUND_SU2, S>(a, dag, has_a, norm, full, st, clov);
        default: return dispatch_hop_clov<HRD_ADJ_SU2, S>(a, dag, has_a, norm, full, st, clov);
    }
}

}  // namespace

int hop_blocks(const Geom &g) { return (g.Vh + kHopBlock - 1) / kHopBlock; }

int hop_partials(int rep, int prec, const Geom &g)
{
    const int sites = hop_sites_per_block(rep, prec);
    return (g.Vh + sites - 1) / sites;
}

// Whether every spinor and link block an FP64 hop of this geometry reads is
// below 2 GiB, so that 32-bit offsets from the block bases address it.
bool blocks_fit_32(int rep, const Geom &g)
{
    const long long lim = 1ll << 31;
    return (long long)g.Vh * spinor_site_bytes(rep, HRD_F64) < lim && (long long)g.Vh * link_bytes(rep, HRD_F64) < lim;
}

hipError_t launch_hop_rupdate(int rep, int prec, const HopArgs &a0, hipStream_t st, int clov)
{
    if (is_dense(rep)) return launch_hop_rupdate_dense(rep, prec, a0, st, clov);
    HopArgs a = a0;
    a.rel = prec == HRD_F64 && blocks_fit_32(rep, a.g);
    switch (prec) {
        case HRD_F64: return rupd_for<double>(rep, a, st, clov);
        case HRD_F32: return rupd_for<float>(rep, a, st, clov);
        default: return rupd_for<h16>(rep, a, st, clov);
    }
}

hipError_t launch_hop(int rep, int prec, const HopArgs &a0, bool dag, bool has_a, bool norm, bool full,
                      hipStream_t st, int clov)
{
    if (is_dense(rep)) return launch_hop_dense(rep, prec, a0, dag, has_a, norm, full, st, clov);
    HopArgs a = a0;
    a.rel = prec == HRD_F64 && blocks_fit_32(rep, a.g);
    switch (prec) {
        case HRD_F64: return hop_for<double>(rep, a, dag, has_a, norm, full, st, clov);
        case HRD_F32: return hop_for<float>(rep, a, dag, has_a, norm, full, st, clov);
        default: return hop_for<h16>(rep, a, dag, has_a, norm, full, st, clov);
    }
}

}  // namespace hrd
