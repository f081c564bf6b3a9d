// Precision-dependent launchers of the dense kernels.  This file is compiled
// once per contraction precision (-DGLRM_PREC=<0|1|3>: FP32, split BF16, plain
// BF16) and loss set (-DGLRM_LKS=<0|1>: the quadratic loss everywhere, or a
// per-column loss table), so the instances build in parallel and each set can
// get its own code-generation flags.  The launchers that do not depend on the
// loss are built with the loss-table set.
#include <type_traits>

#include "dense_kernels.h"

#ifndef GLRM_PREC
#error "compile with -DGLRM_PREC=0, 1 or 3"
#endif
#ifndef GLRM_LKS
#error "compile with -DGLRM_LKS=0 (quadratic) or 1 (loss table)"
#endif

namespace glrm {

#define GLRM_DISPATCH_KP(KPV, ...)                                    \
    switch (KPV) {                                                    \
    case 16: { constexpr int KP = 16; __VA_ARGS__; } break;           \
    case 32: { constexpr int KP = 32; __VA_ARGS__; } break;           \
    case 64: { constexpr int KP = 64; __VA_ARGS__; } break;           \
    default: return hipErrorInvalidValue;                              \
    }
#define GLRM_DISPATCH_PREC(PV, ...)                                   \
    switch (PV) {                                                     \
    case P_FP32: { constexpr int PREC = P_FP32; __VA_ARGS__; } break; \
    case P_BF16: { constexpr int PREC = P_BF16; __VA_ARGS__; } break; \
    case P_BF16_PLAIN: { constexpr int PREC = P_BF16_PLAIN; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                              \
    }
#define GLRM_DISPATCH_TPW(TV, ...)                                    \
    switch (TV) {                                                     \
    case 1: { constexpr int TPW = 1; __VA_ARGS__; } break;            \
    case 2: { constexpr int TPW = 2; __VA_ARGS__; } break;            \
    case 4: { constexpr int TPW = 4; __VA_ARGS__; } break;            \
    case 8: { constexpr int TPW = 8; __VA_ARGS__; } break;            \
    default: return hipErrorInvalidValue;                              \
    }

// Up to 16 tiles per wavefront (the fused row pass at kp <= 32).
#define GLRM_DISPATCH_TPW16(TV, ...)                                  \
    switch (TV) {                                                     \
    case 1: { constexpr int TPW = 1; __VA_ARGS__; } break;            \
    case 2: { constexpr int TPW = 2; __VA_ARGS__; } break;            \
    case 4: { constexpr int TPW = 4; __VA_ARGS__; } break;            \
    case 8: { constexpr int TPW = 8; __VA_ARGS__; } break;            \
    case 16: { constexpr int TPW = 16; __VA_ARGS__; } break;          \
    default: return hipErrorInvalidValue;                              \
    }

// The loss instance of a loss set: the quadratic loss (every column) gets its
// own instances; a loss table goes through the per-tile loss selection.
template <int LKS>
constexpr int LK_OF = LKS == 0 ? L_QUAD : -1;

// Calls f(KP, TPW) as integral constants for the runtime values (TPW up to 16).
template <typename F>
static void for_instance(int kp, int tpw, F &&f)
{
    auto with_tpw = [&](auto kpc) {
        switch (tpw) {
        case 1: f(kpc, std::integral_constant<int, 1>{}); break;
        case 2: f(kpc, std::integral_constant<int, 2>{}); break;
        case 4: f(kpc, std::integral_constant<int, 4>{}); break;
        case 8: f(kpc, std::integral_constant<int, 8>{}); break;
        case 16: f(kpc, std::integral_constant<int, 16>{}); break;
        default: break;
        }
    };
    switch (kp) {
    case 16: with_tpw(std::integral_constant<int, 16>{}); break;
    case 32: with_tpw(std::integral_constant<int, 32>{}); break;
    case 64: with_tpw(std::integral_constant<int, 64>{}); break;
    default: break;
    }
}

template <int PREC, int LKS>
hipError_t launch_xstep_p(const XStepArgs &a, int kp, int tpw, int grid, hipStream_t st)
{
    constexpr int LK = LK_OF<LKS>;
    GLRM_DISPATCH_KP(kp, GLRM_DISPATCH_TPW16(tpw,
        if constexpr (KP == 64 && TPW == 16) return hipErrorInvalidValue;
        else hipLaunchKernelGGL((xstep_kernel<KP, TPW, PREC, LK>), dim3(grid), dim3(NTX_OF<KP>), 0, st, a)));
    return hipGetLastError();
}

// Workgroups of one instance that fit on a CU at once (registers and LDS).
template <typename K>
static int blocks_per_cu(K kernel, int threads)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) return 1;
    return nb;
}

template <int PREC, int LKS>
int xstep_blocks_p(int kp, int tpw)
{
    constexpr int LK = LK_OF<LKS>;
    int nb = 1;
    auto pick = [&](auto kpc, auto tpwc) {
        constexpr int KP = decltype(kpc)::value, TPW = decltype(tpwc)::value;
        if constexpr (!(KP == 64 && TPW == 16)) nb = blocks_per_cu(xstep_kernel<KP, TPW, PREC, LK>, NTX_OF<KP>);
    };
    for_instance(kp, tpw, pick);
    return nb;
}

template <int PREC, int LKS>
int ycheck_blocks_p(int kp, int tpw)
{
    constexpr int LK = LK_OF<LKS>;
    int nb = 1;
    auto pick = [&](auto kpc, auto tpwc) {
        constexpr int KP = decltype(kpc)::value, TPW = decltype(tpwc)::value;
        if constexpr (TPW <= 8) nb = blocks_per_cu(ycheck_kernel<KP, TPW, PREC, LK>, NTY_OF<KP>);
    };
    for_instance(kp, tpw, pick);
    return nb;
}

template <int PREC, int LKS>
hipError_t launch_ycheck_p(const YCheckArgs &a, int kp, int tpw, int grid, hipStream_t st)
{
    constexpr int LK = LK_OF<LKS>;
    GLRM_DISPATCH_KP(kp, GLRM_DISPATCH_TPW(tpw,
        hipLaunchKernelGGL((ycheck_kernel<KP, TPW, PREC, LK>), dim3(grid), dim3(NTY_OF<KP>), 0, st, a)));
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_yprox_p(const YProxArgs &a, int kp, hipStream_t st)
{
    const int blocks = (int)((a.n * (int64_t)kp + 63) / 64);
    GLRM_DISPATCH_KP(kp, hipLaunchKernelGGL((yprox_kernel<KP, PREC>), dim3(blocks), dim3(64 * YPROX_SPLIT), 0, st, a));
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_yaccept_p(const YAcceptArgs &a, int kp, int blocks, hipStream_t st)
{
    GLRM_DISPATCH_KP(kp, hipLaunchKernelGGL((yaccept_kernel<KP, PREC>), dim3(blocks), dim3(256), 0, st, a));
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_yshadow_p(const YShadowArgs &a, int kp, hipStream_t st)
{
    const int blocks = (int)((a.ldp * (int64_t)kp + 255) / 256);
    GLRM_DISPATCH_KP(kp, hipLaunchKernelGGL((yshadow_kernel<KP, PREC>), dim3(blocks), dim3(256), 0, st, a));
    return hipGetLastError();
}

template <int PREC, int LKS>
hipError_t launch_lossgrad_p(const LossGradArgs &a, int kp, int tpw, bool want_grad, int gx, int gy, hipStream_t st)
{
    constexpr int LK = LK_OF<LKS>;
    if (want_grad) {
        GLRM_DISPATCH_KP(kp, GLRM_DISPATCH_TPW16(tpw,
            if constexpr (KP == 64 && TPW > 2) return hipErrorInvalidValue;
            else hipLaunchKernelGGL((lossgrad_kernel<KP, TPW, PREC, LK, true>), dim3(gx, gy), dim3(NTG_OF<KP>), 0, st,
                                    a)));
    } else {
        GLRM_DISPATCH_KP(kp, GLRM_DISPATCH_TPW16(tpw,
            if constexpr (KP == 64 && TPW > 2) return hipErrorInvalidValue;
            else hipLaunchKernelGGL((lossgrad_kernel<KP, TPW, PREC, LK, false>), dim3(gx, gy), dim3(NTG_OF<KP>), 0, st,
                                    a)));
    }
    return hipGetLastError();
}

// The column-blocked row half-step: 16 tiles per wavefront at kp <= 32, 4 at
// kp = 64 (the gradient pass's widest instances, which tables too wide for
// the fused row pass always take).
template <int PREC, int LKS>
hipError_t launch_xwide_p(const XWideArgs &a, int mode, int kp, int tpw, int gx, int gy, hipStream_t st)
{
    constexpr int LK = LK_OF<LKS>;
    auto go = [&](auto kpc, auto tpwc) -> hipError_t {
        constexpr int KP = decltype(kpc)::value, TPW = decltype(tpwc)::value;
        switch (mode) {
        case 0: hipLaunchKernelGGL((xwide_kernel<KP, TPW, PREC, LK, 0>), dim3(gx, gy), dim3(NTX_OF<KP>), 0, st, a); break;
        case 1: hipLaunchKernelGGL((xwide_kernel<KP, TPW, PREC, LK, 1>), dim3(gx, gy), dim3(NTX_OF<KP>), 0, st, a); break;
        case 2: hipLaunchKernelGGL((xwide_kernel<KP, TPW, PREC, LK, 2>), dim3(gx, gy), dim3(NTX_OF<KP>), 0, st, a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    };
    if (kp == 16 && tpw == 16) return go(std::integral_constant<int, 16>{}, std::integral_constant<int, 16>{});
    if (kp == 32 && tpw == 16) return go(std::integral_constant<int, 32>{}, std::integral_constant<int, 16>{});
    if (kp == 64 && tpw == 4) return go(std::integral_constant<int, 64>{}, std::integral_constant<int, 4>{});
    return hipErrorInvalidValue;
}

// Workgroups of the column pass (mode 2) that fit on a CU.
template <int PREC, int LKS>
int xwide_blocks_p(int kp, int tpw)
{
    constexpr int LK = LK_OF<LKS>;
    if (kp == 16 && tpw == 16) return blocks_per_cu(xwide_kernel<16, 16, PREC, LK, 2>, NTX_OF<16>);
    if (kp == 32 && tpw == 16) return blocks_per_cu(xwide_kernel<32, 16, PREC, LK, 2>, NTX_OF<32>);
    if (kp == 64 && tpw == 4) return blocks_per_cu(xwide_kernel<64, 4, PREC, LK, 2>, NTX_OF<64>);
    return 1;
}

template hipError_t launch_xwide_p<GLRM_PREC, GLRM_LKS>(const XWideArgs &, int, int, int, int, int, hipStream_t);
template int xwide_blocks_p<GLRM_PREC, GLRM_LKS>(int, int);
template hipError_t launch_xstep_p<GLRM_PREC, GLRM_LKS>(const XStepArgs &, int, int, int, hipStream_t);
template int xstep_blocks_p<GLRM_PREC, GLRM_LKS>(int, int);
template int ycheck_blocks_p<GLRM_PREC, GLRM_LKS>(int, int);
template hipError_t launch_ycheck_p<GLRM_PREC, GLRM_LKS>(const YCheckArgs &, int, int, int, hipStream_t);
template hipError_t launch_lossgrad_p<GLRM_PREC, GLRM_LKS>(const LossGradArgs &, int, int, bool, int, int,
                                                           hipStream_t);
#if GLRM_LKS == 1
template hipError_t launch_yprox_p<GLRM_PREC>(const YProxArgs &, int, hipStream_t);
template hipError_t launch_yaccept_p<GLRM_PREC>(const YAcceptArgs &, int, int, hipStream_t);
template hipError_t launch_yshadow_p<GLRM_PREC>(const YShadowArgs &, int, hipStream_t);
#endif

}  // namespace glrm
