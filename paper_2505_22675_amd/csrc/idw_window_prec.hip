// Window-form IDW, precision variants (FP16 tile-relative offsets, FP32
// absolute coordinates).  Membership, ranking and weights come from the
// variant's FP32 squared distance; the ranking key is its bit pattern, which
// always fits the packed 64-bit (key, index) form.
#include "idw_window_impl.hpp"

namespace auv {

using namespace win;

auv_status launch_idw_window_prec(const auv_bin_view &bv, const IdwArgs &a, const WinGeom &g,
                                  int pmode, hipStream_t st)
{
    const int ntx = (a.nx + kTW - 1) / kTW, nty = (a.ny + kTH - 1) / kTH;
    const bool nn = (a.mode & 2) != 0;
    if (!(a.mode & 1))
        return fail(AUV_ERR_INVALID, "precision variants apply to IDW only");
    if (a.precision == AUV_P_FP16_OFFSETS) {
        if (nn)
            launch_mode<3, true, AUV_P_FP16_OFFSETS>(bv, a, g, ntx, nty, pmode, st);
        else
            launch_mode<1, true, AUV_P_FP16_OFFSETS>(bv, a, g, ntx, nty, pmode, st);
    } else if (a.precision == AUV_P_FP32_ABSOLUTE) {
        if (nn)
            launch_mode<3, true, AUV_P_FP32_ABSOLUTE>(bv, a, g, ntx, nty, pmode, st);
        else
            launch_mode<1, true, AUV_P_FP32_ABSOLUTE>(bv, a, g, ntx, nty, pmode, st);
    } else {
        return fail(AUV_ERR_INVALID, "unknown precision variant");
    }
    AUV_HIP(hipGetLastError());
    return AUV_OK;
}

}  // namespace auv
