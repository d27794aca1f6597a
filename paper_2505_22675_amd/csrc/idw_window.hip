// Window-form IDW: launchers of the exact lattice path, the window geometry
// and the dispatch to the precision variants (idw_window_prec.hip).  The
// kernel itself is in idw_window_impl.hpp.
#include "idw_span_impl.hpp"

#include <cmath>

namespace auv {

using namespace win;

bool window_geometry(const IdwArgs &a, WinGeom *g)
{
    const double DX = a.dx * kLatticePerMetre, DY = a.dy * kLatticePerMetre;
    // linear node lattice: (b + 1/2) * DX must be an integer for every b
    if (DX != std::floor(DX) || DY != std::floor(DY) || std::fmod(DX, 2.0) != 0.0 ||
        std::fmod(DY, 2.0) != 0.0 || DX >= 2147483648.0 || DY >= 2147483648.0)
        return false;
    g->DXl = (int)DX;
    g->DYl = (int)DY;
    g->X0 = g->DXl / 2;
    g->Y0 = g->DYl / 2;
    // window offsets stay within +-2^22 lattice units (the kernel's exact
    // squares use 24-bit multiplies): reach below 32 m
    if (a.R_stage >= (1 << 21))
        return false;
    g->Wx = (int)((2LL * a.R_stage) / g->DXl) + 1;
    g->Wy = (int)((2LL * a.R_stage) / g->DYl) + 1;
    if ((long long)g->Wx * g->Wy > 64LL * kMaxChunks)
        return false;
    g->ncells = g->Wx * g->Wy;
    g->nchunks = (g->ncells + 63) / 64;
    // jb/ia are packed as 16-bit fields of one word
    if (g->Wx > 30000 || g->Wy > 30000)
        return false;
    return true;
}

auv_status launch_idw_window(const auv_bin_view &bv, const IdwArgs &a, const WinGeom &g,
                             int pmode, hipStream_t st)
{
    const int TH = tile_rows(a);
    const int ntx = (a.nx + kTW - 1) / kTW, nty = (a.ny + TH - 1) / TH;
    if (a.precision != AUV_P_FP32_REBASE)
        return launch_idw_window_prec(bv, a, g, pmode, st);
    if (a.span && span::span_ok(bv, a, g, pmode)) {
        switch (a.mode) {
        case 1: span::launch_shape<1, 16, 16>(bv, a, g, pmode, st); break;
        case 2: span::launch_shape<2, 16, 16>(bv, a, g, pmode, st); break;
        default: span::launch_shape<3, 16, 16>(bv, a, g, pmode, st); break;
        }
        AUV_HIP(hipGetLastError());
        return AUV_OK;
    }
    switch (a.mode) {
    case 1: launch_mode<1, AUV_P_FP32_REBASE>(bv, a, g, ntx, nty, pmode, st); break;
    case 2: launch_mode<2, AUV_P_FP32_REBASE>(bv, a, g, ntx, nty, pmode, st); break;
    case 3: launch_mode<3, AUV_P_FP32_REBASE>(bv, a, g, ntx, nty, pmode, st); break;
    default: return fail(AUV_ERR_INVALID, "bad IDW mode");
    }
    AUV_HIP(hipGetLastError());
    return AUV_OK;
}

}  // namespace auv
