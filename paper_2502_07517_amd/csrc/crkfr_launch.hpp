// Host-side launchers of the templated kernels for one equation.  Each
// equation's translation unit instantiates these for N = 1..4, FP64 and MP32.
#pragma once
#include "crkfr_kernels.hpp"

namespace crkfr {

enum { PH_LOCAL = 0, PH_FACE_X = 1, PH_FACE_Y = 2, PH_UPDATE = 3, PH_IMPORT = 4, PH_EXPORT = 5, PH_GHOST = 6,
       PH_FEATURES = 7, PH_STATS = 8, PH_TILE = 9, PH_TILE_FACE_X = 10, PH_TILE_FACE_Y = 11, PH_EDGE_UPDATE = 12,
       PH_UPDATE_FU = 13, PH_CB_LOCAL = 14, PH_CB_WHITE = 15, PH_CB_UPDATE = 16,
       // the update phases in one-wavefront workgroups (elements of 16 points;
       // elsewhere the same launch as the phase without _W)
       PH_UPDATE_W = 17, PH_UPDATE_FU_W = 18, PH_CB_UPDATE_W = 19 };

template <template <class> class EqT, int N, class real, bool LIM>
static int launch_step_phase(int phase, const StepArgs<real>& a, hipStream_t st)
{
    using Eq = EqT<real>;
    using G = Geo<Eq::DIM, N>;
    const int nb = (a.ne + G::EB - 1) / G::EB;
    switch (phase) {
    case PH_LOCAL: {
        using LG = LGeo<Eq::DIM, N>;
        const int nbl = (a.ne + LG::EB - 1) / LG::EB;
        hipLaunchKernelGGL((k_local<Eq, N, real, LIM>), dim3(nbl), dim3(LG::BLOCK), 0, st, a);
        break;
    }
    case PH_FACE_X: {
        long long tot = (long long)a.ny * (a.nx + 1) * G::nq;
        hipLaunchKernelGGL((k_face<Eq, N, real, LIM, 0>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a);
        break;
    }
    case PH_FACE_Y:
        if constexpr (Eq::DIM == 2) {
            long long tot = (long long)(a.ny + 1) * a.nx * G::nd;
            hipLaunchKernelGGL((k_face<Eq, N, real, LIM, 1>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a);
        }
        break;
    case PH_UPDATE:
        hipLaunchKernelGGL((k_update<Eq, N, real, LIM>), dim3(nb), dim3(G::BLOCK), 0, st, a);
        break;
    case PH_UPDATE_FU:
        hipLaunchKernelGGL((k_update<Eq, N, real, LIM, true>), dim3(nb), dim3(G::BLOCK), 0, st, a);
        break;
    case PH_FEATURES:
        hipLaunchKernelGGL((k_features<Eq, N, real>), dim3(nb), dim3(G::BLOCK), 0, st, a);
        break;
    case PH_TILE:
    case PH_TILE_FACE_X:
    case PH_TILE_FACE_Y:
        // the tile-fused step: Euler 2D, elements of 4 or 16 points, limiter off
        if constexpr (TGeo<Eq::DIM, N, (int)sizeof(real)>::OK && Eq::ID == 2 && !LIM) {
            using TG = TGeo<Eq::DIM, N, (int)sizeof(real)>;
            const int ntx = (a.nx + TG::TX - 1) / TG::TX, nty = (a.ny + TG::TY - 1) / TG::TY;
            if (phase == PH_TILE) {
                hipLaunchKernelGGL((k_tile<Eq, N, real>), dim3(ntx * nty), dim3(TG::BLOCK), 0, st, a);
            } else if (phase == PH_TILE_FACE_X) {
                long long tot = (long long)a.ny * (ntx + 1) * G::nq;
                hipLaunchKernelGGL((k_tile_face<Eq, N, real, 0>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                                   st, a);
            } else {
                long long tot = (long long)(nty + 1) * a.nx * G::nd;
                hipLaunchKernelGGL((k_tile_face<Eq, N, real, 1>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                                   st, a);
            }
            return 0;
        }
        return -1;
    case PH_CB_LOCAL:
    case PH_CB_WHITE:
    case PH_CB_UPDATE:
        // the checkerboard step: 2D, limiter off, half the elements per launch
        if constexpr (Eq::DIM == 2 && !LIM) {
            using LG = LGeo<Eq::DIM, N>;
            const int nc = a.ne / 2;
            if (phase == PH_CB_LOCAL)
                hipLaunchKernelGGL((k_cb_local<Eq, N, real>), dim3((nc + LG::EB - 1) / LG::EB), dim3(LG::BLOCK), 0, st, a);
            else if (phase == PH_CB_WHITE)
                hipLaunchKernelGGL((k_cb_white<Eq, N, real>), dim3((nc + LG::EB - 1) / LG::EB), dim3(LG::BLOCK), 0, st, a);
            else
                hipLaunchKernelGGL((k_cb_update<Eq, N, real>), dim3((nc + G::EB - 1) / G::EB), dim3(G::BLOCK), 0, st, a);
            return 0;
        }
        return -1;
    case PH_EDGE_UPDATE:
        hipLaunchKernelGGL((k_update<Eq, N, real, LIM>), dim3((a.n_edge + G::EB - 1) / G::EB), dim3(G::BLOCK), 0,
                           st, a);
        break;
    case PH_UPDATE_W:
    case PH_UPDATE_FU_W:
    case PH_CB_UPDATE_W:
        if constexpr (G::np == 16) {
            using GW = UGeo<Eq::DIM, N, 1>;
            if (phase == PH_UPDATE_W) {
                hipLaunchKernelGGL((k_update<Eq, N, real, LIM, false, 1>), dim3((a.ne + GW::EB - 1) / GW::EB),
                                   dim3(GW::BLOCK), 0, st, a);
            } else if (phase == PH_UPDATE_FU_W) {
                hipLaunchKernelGGL((k_update<Eq, N, real, LIM, true, 1>), dim3((a.ne + GW::EB - 1) / GW::EB),
                                   dim3(GW::BLOCK), 0, st, a);
            } else {
                if constexpr (Eq::DIM == 2 && !LIM) {
                    const int nc = a.ne / 2;
                    hipLaunchKernelGGL((k_cb_update<Eq, N, real, 1>), dim3((nc + GW::EB - 1) / GW::EB),
                                       dim3(GW::BLOCK), 0, st, a);
                } else {
                    return -1;
                }
            }
            return 0;
        } else {
            return launch_step_phase<EqT, N, real, LIM>(
                phase == PH_UPDATE_W ? PH_UPDATE : (phase == PH_UPDATE_FU_W ? PH_UPDATE_FU : PH_CB_UPDATE), a, st);
        }
    }
    return 0;
}

template <template <class> class EqT, int N, class real>
static void launch_io_phase(int phase, const IoArgs<real>& a, hipStream_t st)
{
    using Eq = EqT<real>;
    using G = Geo<Eq::DIM, N>;
    const int nb = (a.ne + G::EB - 1) / G::EB;
    switch (phase) {
    case PH_IMPORT:
        hipLaunchKernelGGL((k_import<Eq, N, real>), dim3(nb), dim3(G::BLOCK), 0, st, a);
        break;
    case PH_EXPORT:
        hipLaunchKernelGGL((k_export<Eq, N, real>), dim3(nb), dim3(G::BLOCK), 0, st, a);
        break;
    case PH_STATS:
        hipLaunchKernelGGL((k_stats<Eq, N, real>), dim3(nb), dim3(G::BLOCK), 0, st, a);
        break;
    case PH_GHOST: {
        int tot = 2 * a.ny * G::nq + (Eq::DIM == 2 ? 2 * a.nx * G::nd : 0);
        hipLaunchKernelGGL((k_ghost<Eq, N, real>), dim3((tot + 255) / 256), dim3(256), 0, st, a);
        break;
    }
    }
}

// work-item block sizes of each phase (host side)
template <template <class> class EqT, int N, class real>
static void batch_geometry(int* elems_local, int* elems_update, int* nq)
{
    using Eq = EqT<real>;
    *elems_local = LGeo<Eq::DIM, N>::EB;
    *elems_update = Geo<Eq::DIM, N>::EB;
    *nq = Geo<Eq::DIM, N>::nq;
}

template <template <class> class EqT, int N, class real, bool LIM>
static void launch_batch_phase(int phase, const StepArgs<real>* args, const int2* work, int nwork, int grid,
                               hipStream_t st)
{
    using Eq = EqT<real>;
    const dim3 g(grid > 0 ? grid : nwork);
    const int bl = phase == BPH_LOCAL ? LGeo<Eq::DIM, N>::BLOCK
                 : (phase == BPH_UPDATE || phase == BPH_UPDATE_FU ? Geo<Eq::DIM, N>::BLOCK : 256);
#define CRKFR_BATCH_LAUNCH(PH)                                                                        \
    if (grid > 0)                                                                                     \
        hipLaunchKernelGGL((k_batch_persistent<Eq, N, real, LIM, PH>), g, dim3(bl), 0, st, args, work, nwork); \
    else                                                                                              \
        hipLaunchKernelGGL((k_batch<Eq, N, real, LIM, PH>), g, dim3(bl), 0, st, args, work, nwork);
    switch (phase) {
    case BPH_LOCAL: CRKFR_BATCH_LAUNCH(BPH_LOCAL) break;
    case BPH_FACE_X: CRKFR_BATCH_LAUNCH(BPH_FACE_X) break;
    case BPH_FACE_Y:
        if constexpr (Eq::DIM == 2) { CRKFR_BATCH_LAUNCH(BPH_FACE_Y) }
        break;
    case BPH_UPDATE: CRKFR_BATCH_LAUNCH(BPH_UPDATE) break;
    case BPH_UPDATE_FU: CRKFR_BATCH_LAUNCH(BPH_UPDATE_FU) break;
    }
#undef CRKFR_BATCH_LAUNCH
}

template <template <class> class EqT, class real>
static int launch_batch(int N, bool lim, int phase, const StepArgs<real>* args, const int2* work, int nwork,
                        int grid, hipStream_t st)
{
#define CRKFR_BCASE(NN)                                                                           \
    case NN:                                                                                      \
        if (lim) launch_batch_phase<EqT, NN, real, true>(phase, args, work, nwork, grid, st);     \
        else launch_batch_phase<EqT, NN, real, false>(phase, args, work, nwork, grid, st);        \
        return 0;
    switch (N) {
        CRKFR_BCASE(1)
        CRKFR_BCASE(2)
        CRKFR_BCASE(3)
        CRKFR_BCASE(4)
    }
#undef CRKFR_BCASE
    return -1;
}

// tile of the tile-fused step (elements per direction), -1 when there is none
template <template <class> class EqT, int N, class real>
static int tile_shape_n(int* tx, int* ty)
{
    using Eq = EqT<real>;
    using TG = TGeo<Eq::DIM, N, (int)sizeof(real)>;
    if constexpr (TG::OK && Eq::ID == 2) {
        *tx = TG::TX;
        *ty = TG::TY;
        return 0;
    }
    return -1;
}

template <template <class> class EqT>
static int tile_shape(int N, int mp, int* tx, int* ty)
{
    switch (N) {
    case 1: return mp ? tile_shape_n<EqT, 1, float>(tx, ty) : tile_shape_n<EqT, 1, double>(tx, ty);
    case 2: return mp ? tile_shape_n<EqT, 2, float>(tx, ty) : tile_shape_n<EqT, 2, double>(tx, ty);
    case 3: return mp ? tile_shape_n<EqT, 3, float>(tx, ty) : tile_shape_n<EqT, 3, double>(tx, ty);
    case 4: return mp ? tile_shape_n<EqT, 4, float>(tx, ty) : tile_shape_n<EqT, 4, double>(tx, ty);
    }
    return -1;
}

template <template <class> class EqT, class real>
static int geometry(int N, int* el, int* eu, int* nq)
{
    switch (N) {
    case 1: batch_geometry<EqT, 1, real>(el, eu, nq); return 0;
    case 2: batch_geometry<EqT, 2, real>(el, eu, nq); return 0;
    case 3: batch_geometry<EqT, 3, real>(el, eu, nq); return 0;
    case 4: batch_geometry<EqT, 4, real>(el, eu, nq); return 0;
    }
    return -1;
}

template <template <class> class EqT, class real>
static int launch_step(int N, bool lim, int phase, const StepArgs<real>& a, hipStream_t st)
{
#define CRKFR_CASE(NN)                                                            \
    case NN:                                                                      \
        if (lim) return launch_step_phase<EqT, NN, real, true>(phase, a, st);     \
        return launch_step_phase<EqT, NN, real, false>(phase, a, st);
    switch (N) {
        CRKFR_CASE(1)
        CRKFR_CASE(2)
        CRKFR_CASE(3)
        CRKFR_CASE(4)
    }
#undef CRKFR_CASE
    return -1;
}

template <template <class> class EqT, class real>
static int launch_io(int N, int phase, const IoArgs<real>& a, hipStream_t st)
{
    switch (N) {
    case 1: launch_io_phase<EqT, 1, real>(phase, a, st); return 0;
    case 2: launch_io_phase<EqT, 2, real>(phase, a, st); return 0;
    case 3: launch_io_phase<EqT, 3, real>(phase, a, st); return 0;
    case 4: launch_io_phase<EqT, 4, real>(phase, a, st); return 0;
    }
    return -1;
}

// type-erased entry points, one set per equation (defined in crkfr_eq_*.hip)
#define CRKFR_DECLARE_EQ(name)                                                                      \
    int name##_step_f64(int N, bool lim, int phase, const StepArgs<double>& a, hipStream_t st);    \
    int name##_step_f32(int N, bool lim, int phase, const StepArgs<float>& a, hipStream_t st);     \
    int name##_io_f64(int N, int phase, const IoArgs<double>& a, hipStream_t st);                  \
    int name##_io_f32(int N, int phase, const IoArgs<float>& a, hipStream_t st);                   \
    int name##_batch_f64(int N, bool lim, int phase, const StepArgs<double>* args, const int2* work, \
                         int nwork, int grid, hipStream_t st);                                     \
    int name##_batch_f32(int N, bool lim, int phase, const StepArgs<float>* args, const int2* work,  \
                         int nwork, int grid, hipStream_t st);                                     \
    int name##_geometry(int N, int* elems_local, int* elems_update, int* nq);                      \
    int name##_tile_shape(int N, int mp, int* tx, int* ty);
#define CRKFR_DEFINE_EQ(name, EqT)                                                                  \
    int name##_step_f64(int N, bool lim, int phase, const StepArgs<double>& a, hipStream_t st)     \
    { return launch_step<EqT, double>(N, lim, phase, a, st); }                                      \
    int name##_step_f32(int N, bool lim, int phase, const StepArgs<float>& a, hipStream_t st)      \
    { return launch_step<EqT, float>(N, lim, phase, a, st); }                                       \
    int name##_io_f64(int N, int phase, const IoArgs<double>& a, hipStream_t st)                   \
    { return launch_io<EqT, double>(N, phase, a, st); }                                             \
    int name##_io_f32(int N, int phase, const IoArgs<float>& a, hipStream_t st)                    \
    { return launch_io<EqT, float>(N, phase, a, st); }                                              \
    int name##_batch_f64(int N, bool lim, int phase, const StepArgs<double>* args, const int2* work, \
                         int nwork, int grid, hipStream_t st)                                      \
    { return launch_batch<EqT, double>(N, lim, phase, args, work, nwork, grid, st); }               \
    int name##_batch_f32(int N, bool lim, int phase, const StepArgs<float>* args, const int2* work,  \
                         int nwork, int grid, hipStream_t st)                                      \
    { return launch_batch<EqT, float>(N, lim, phase, args, work, nwork, grid, st); }                \
    int name##_geometry(int N, int* el, int* eu, int* nq) { return geometry<EqT, double>(N, el, eu, nq); }   \
    int name##_tile_shape(int N, int mp, int* tx, int* ty) { return tile_shape<EqT>(N, mp, tx, ty); }

CRKFR_DECLARE_EQ(linadv1d)
CRKFR_DECLARE_EQ(euler1d)
CRKFR_DECLARE_EQ(euler2d)
CRKFR_DECLARE_EQ(tenmom2d)
CRKFR_DECLARE_EQ(burgers1d)
CRKFR_DECLARE_EQ(tenmom1d)

}  // namespace crkfr
