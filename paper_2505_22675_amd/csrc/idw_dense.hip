// Dense IDW form: launcher.  The per-tile code is in idw_dense_impl.hpp.
#include "idw_dense_impl.hpp"

namespace auv {

using namespace dense;

namespace {

template <int kMode>
void launch_k(const auv_bin_view &bv, const IdwArgs &a, int ntx, int nty, int pmode,
              hipStream_t st)
{
    const dim3 grid((unsigned)(ntx * nty)), block(64);
    if (a.max_pts <= 16)
        k_idw_dense<kMode, 16><<<grid, block, 0, st>>>(bv, a, ntx, nty, pmode);
    else
        k_idw_dense<kMode, 32><<<grid, block, 0, st>>>(bv, a, ntx, nty, pmode);
}

}  // namespace

auv_status launch_idw_dense(const auv_bin_view &bv, const IdwArgs &a, int pmode,
                            hipStream_t st)
{
    if (a.max_pts < 1 || a.max_pts > 32)
        return fail(AUV_ERR_INVALID, "the dense form needs 1 <= max_pts <= 32");
    if (!dense_key_ok(a.R, bv.idx_bits))
        return fail(AUV_ERR_RANGE, "the dense form needs (R^2 << index bits) below 2^62");
    const int TW = dense_tile_w(a), TH = 64 / TW;
    const int ntx = (a.nx + TW - 1) / TW, nty = (a.ny + TH - 1) / TH;
    switch (a.mode) {
    case 1: launch_k<1>(bv, a, ntx, nty, pmode, st); break;
    case 2: launch_k<2>(bv, a, ntx, nty, pmode, st); break;
    case 3: launch_k<3>(bv, a, ntx, nty, pmode, st); break;
    default: return fail(AUV_ERR_INVALID, "bad IDW mode");
    }
    AUV_HIP(hipGetLastError());
    return AUV_OK;
}

}  // namespace auv
