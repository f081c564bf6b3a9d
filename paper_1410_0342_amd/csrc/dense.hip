// Dense-layout kernels that do not depend on the contraction precision, and
// the launch dispatch (the precision-dependent kernels are instantiated in
// dense_prec.hip, one translation unit per precision).
#include "dense_kernels.h"

namespace glrm {

// One workgroup: F = sum of column parts + row regularizers, rejection counts.
__global__ __launch_bounds__(256) void finalize_kernel(FinalizeArgs a)
{
    __shared__ double sF[256];
    __shared__ long long sr[256], sc[256];
    double F = 0.0;
    long long rr = 0, rc = 0;
    for (int q = threadIdx.x; q < a.n_colparts; q += 256) { F += a.part_F[q]; rc += a.part_rejc[q]; }
    for (int q = threadIdx.x; q < a.n_rowparts; q += 256) { F += (double)a.part_rowreg[q]; rr += a.part_rej[q]; }
    sF[threadIdx.x] = F;
    sr[threadIdx.x] = rr;
    sc[threadIdx.x] = rc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sF[threadIdx.x] += sF[threadIdx.x + o];
            sr[threadIdx.x] += sr[threadIdx.x + o];
            sc[threadIdx.x] += sc[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.stats[0] = sF[0];
        a.istats[0] = sr[0];
        a.istats[1] = sc[0];
        if (a.history) a.history[a.sweep] = sF[0];
    }
}

// S4 of the row half-step in column blocks: each row's gradient and loss sum
// over the column blocks (in block order), the prox step to the trial row and
// the regularizer at both.  Sixteen lanes per row, coordinates c0 + 16 q.
__global__ __launch_bounds__(256) void xwide_step_kernel(XWideRowArgs a)
{
    const int ri = threadIdx.x >> 4, c0 = threadIdx.x & 15;
    const int64_t i = (int64_t)blockIdx.x * 16 + ri;
    const bool rv = i < a.m;
    const float al = rv ? a.alpha[i] : 0.0f;
    float rc = 0.0f, rcp = 0.0f;
#pragma unroll
    for (int q = 0; q < GLRM_MAXK_DEV / 16; ++q) {
        const int c = c0 + 16 * q;
        const bool ok = rv && c < a.k;
        float gs = 0.0f, x = 0.0f;
        if (ok) {
            for (int b = 0; b < a.ncb; ++b) gs += a.part_dx[((int64_t)b * a.m + i) * a.k + c];
            x = a.X[i * a.k + c];
        }
        const float xv = ok ? prox_elem(a.rx, al, x - al * gs, c) : 0.0f;
        if (ok) a.Xp[i * a.k + c] = xv;
        rc += ok ? reg_elem(a.rx, x, c) : 0.0f;
        rcp += ok ? reg_elem_trial(a.rx, xv, c) : 0.0f;
    }
    rc = row16_sum(rc);
    rcp = row16_sum(rcp);
    if (c0 == 0 && rv) {
        float f = 0.0f;
        for (int b = 0; b < a.ncb; ++b) f += a.part_f[(int64_t)b * a.mp + i];
        a.rsum[i] = f;
        a.rsum[a.mp + i] = rc;
        a.rsum[2 * a.mp + i] = rcp;
    }
}

// The step rule of the rows (S5): keep the trial row if its objective (loss
// sum over the column blocks, in block order, plus r) does not exceed the
// old one; step sizes move by step_up / step_down.  A fixed grid of 64-row
// groups, so the per-workgroup sums of the decided rows' regularizers and of
// the rejections come in a fixed number and order.
constexpr int XDEC_THREADS = 1024;
__global__ __launch_bounds__(XDEC_THREADS) void xwide_decide_kernel(XWideRowArgs a)
{
    constexpr int NWV = XDEC_THREADS / 64, RPB = XDEC_THREADS / 16;
    __shared__ float s_r[NWV];
    __shared__ int s_j[NWV];
    const int ri = threadIdx.x >> 4, c0 = threadIdx.x & 15;
    float rr = 0.0f;
    int rj = 0;
    for (int64_t p = blockIdx.x; p * RPB < a.m; p += gridDim.x) {
        const int64_t i = p * RPB + ri;
        const bool rv = i < a.m;
        bool acc = false;
        float rx = 0.0f, rxp = 0.0f;
        if (rv) {
            float fp = 0.0f;
            for (int b = 0; b < a.ncb; ++b) fp += a.part_fp[(int64_t)b * a.mp + i];
            rx = a.rsum[a.mp + i];
            rxp = a.rsum[2 * a.mp + i];
            const float f = a.rsum[i] + rx;
            fp += rxp;
            acc = fp <= f;
        }
#pragma unroll
        for (int q = 0; q < GLRM_MAXK_DEV / 16; ++q) {
            const int c = c0 + 16 * q;
            if (acc && c < a.k) a.X[i * a.k + c] = a.Xp[i * a.k + c];
        }
        if (c0 == 0 && rv) {
            const float al = a.alpha[i];
            a.alpha[i] = acc ? al * a.step_up : al * a.step_down;
            rr += acc ? rxp : rx;
            rj += acc ? 0 : 1;
        }
    }
    rr = sum_lanes<64>(rr);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) rj += __shfl_xor(rj, o, 64);
    if ((threadIdx.x & 63) == 0) {
        s_r[threadIdx.x >> 6] = rr;
        s_j[threadIdx.x >> 6] = rj;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = 0.0f;
        int j = 0;
#pragma unroll
        for (int v = 0; v < NWV; ++v) {
            r += s_r[v];
            j += s_j[v];
        }
        a.part_rowreg[blockIdx.x] = r;
        a.part_rej[blockIdx.x] = j;
    }
}

__global__ __launch_bounds__(256) void reduce_dx_kernel(ReduceArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= a.m * a.k) return;
    float s = 0.0f;
    for (int b = 0; b < a.CB; ++b) s += a.part_dx[(int64_t)b * a.m * a.k + t];
    a.dX[t] = s;
}

// FP64 objective: z in double from the fp32 factors, loss in double.  A
// workgroup takes PPB panels of 16 rows x 256 / PPB columns (PPB = 2 for a
// table at most 128 columns wide, so that fewer threads idle past its
// width); each thread owns one column of one panel, keeps y_j in registers
// and reads the panel's 16 x rows as LDS broadcasts.
template <int KP, int PPB>
__global__ __launch_bounds__(256) void objective64_kernel(Obj64Args a)
{
    constexpr int CW = 256 / PPB;              // columns per panel and workgroup
    __shared__ double xsd[PPB][16][KP];
    __shared__ double sred[4];
    const int sub = threadIdx.x / CW, tc = threadIdx.x % CW;
    const int64_t ntile_j = (a.ldp + CW - 1) / CW;
    const int64_t npanels = a.mp / 16, ngroups = (npanels + PPB - 1) / PPB;
    double acc = 0.0;
    for (int64_t blk = blockIdx.x; blk < ngroups * ntile_j; blk += gridDim.x) {
        const int64_t p = (blk / ntile_j) * PPB, jt = blk % ntile_j;
        __syncthreads();
        for (int t = threadIdx.x; t < PPB * 16 * KP; t += 256) {
            const int q = t / (16 * KP), i = (t / KP) % 16, c = t % KP;
            const int64_t row = (p + q) * 16 + i;
            xsd[q][i][c] = (p + q < npanels && row < a.m && c < a.k) ? (double)a.X[row * a.k + c] : 0.0;
        }
        __syncthreads();
        const int64_t i0 = (p + sub) * 16, j = jt * CW + tc;
        if (p + sub < npanels && j < a.n) {
            float avs[16];   // the column's 16 entries, all loads in flight at once
#pragma unroll
            for (int ii = 0; ii < 16; ++ii) avs[ii] = a.Ap[(i0 + ii) * a.ldp + j];
            double y[KP];
#pragma unroll
            for (int c = 0; c < KP; ++c) y[c] = c < a.k ? (double)a.Y[j * a.k + c] : 0.0;
            const int q = a.lt.uniform >= 0 ? a.lt.uniform : a.codes[j];
            const int kind = a.lt.kind[q], lev = a.lt.levels[q];
            const double par = (double)a.lt.param[q];
            const double wj = a.lt.colw ? (double)a.lt.colw[j] : 1.0;
#pragma unroll
            for (int ii = 0; ii < 16; ++ii) {
                const float av = avs[ii];
                if (i0 + ii < a.m && av == av) {
                    double z = 0.0;
#pragma unroll
                    for (int c = 0; c < KP; ++c) z += xsd[sub][ii][c] * y[c];
                    acc += wj * loss_l64(kind, lev, par, z, (double)av);
                }
            }
        }
    }
    acc = sum_lanes64<64>(acc);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) a.part_obj[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// ---------------------------------------------------------------------------
// dispatch by precision (instances live in dense_prec.hip)
// ---------------------------------------------------------------------------
template <int PREC, int LKS> hipError_t launch_xstep_p(const XStepArgs &, int, int, int, hipStream_t);
template <int PREC, int LKS> hipError_t launch_ycheck_p(const YCheckArgs &, int, int, int, hipStream_t);
template <int PREC, int LKS> int xstep_blocks_p(int, int);
template <int PREC, int LKS> int ycheck_blocks_p(int, int);
template <int PREC> hipError_t launch_yprox_p(const YProxArgs &, int, hipStream_t);
template <int PREC> hipError_t launch_yaccept_p(const YAcceptArgs &, int, int, hipStream_t);
template <int PREC> hipError_t launch_yshadow_p(const YShadowArgs &, int, hipStream_t);
template <int PREC, int LKS> hipError_t launch_lossgrad_p(const LossGradArgs &, int, int, bool, int, int, hipStream_t);
template <int PREC, int LKS> hipError_t launch_xwide_p(const XWideArgs &, int, int, int, int, int, hipStream_t);
template <int PREC, int LKS> int xwide_blocks_p(int, int);

#define GLRM_BY_PREC(PV, CALL)                                      \
    switch (PV) {                                                   \
    case P_FP32: return CALL(P_FP32);                               \
    case P_BF16: return CALL(P_BF16);                               \
    case P_BF16_PLAIN: return CALL(P_BF16_PLAIN);                   \
    default: return hipErrorInvalidValue;                           \
    }

// loss set: 0 = the quadratic loss everywhere, 1 = a per-column loss table
static int loss_set(const LossU &lu) { return lu.kind == L_QUAD ? 0 : 1; }

hipError_t launch_xstep(const XStepArgs &a, int kp, int tpw, int prec, int grid, hipStream_t st)
{
    const int lks = loss_set(a.lu);
#define C_(P) (lks == 0 ? launch_xstep_p<P, 0>(a, kp, tpw, grid, st) : launch_xstep_p<P, 1>(a, kp, tpw, grid, st))
    GLRM_BY_PREC(prec, C_)
#undef C_
}

hipError_t launch_ycheck(const YCheckArgs &a, int kp, int tpw, int prec, int grid, hipStream_t st)
{
    const int lks = loss_set(a.lu);
#define C_(P) (lks == 0 ? launch_ycheck_p<P, 0>(a, kp, tpw, grid, st) : launch_ycheck_p<P, 1>(a, kp, tpw, grid, st))
    GLRM_BY_PREC(prec, C_)
#undef C_
}


hipError_t launch_yprox(const YProxArgs &a, int kp, int prec, hipStream_t st)
{
#define C_(P) launch_yprox_p<P>(a, kp, st)
    GLRM_BY_PREC(prec, C_)
#undef C_
}

hipError_t launch_yaccept(const YAcceptArgs &a, int kp, int prec, int blocks, hipStream_t st)
{
#define C_(P) launch_yaccept_p<P>(a, kp, blocks, st)
    GLRM_BY_PREC(prec, C_)
#undef C_
}

int yaccept_blocks(int64_t n, int kp) { return (int)((n * kp + 255) / 256); }

hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_yshadow(const YShadowArgs &a, int kp, int prec, hipStream_t st)
{
#define C_(P) launch_yshadow_p<P>(a, kp, st)
    GLRM_BY_PREC(prec, C_)
#undef C_
}

hipError_t launch_lossgrad(const LossGradArgs &a, int kp, int tpw, int prec, bool want_grad, int gx, int gy,
                           hipStream_t st)
{
    const int lks = loss_set(a.lu);
#define C_(P) (lks == 0 ? launch_lossgrad_p<P, 0>(a, kp, tpw, want_grad, gx, gy, st) \
                        : launch_lossgrad_p<P, 1>(a, kp, tpw, want_grad, gx, gy, st))
    GLRM_BY_PREC(prec, C_)
#undef C_
}

hipError_t launch_xwide(const XWideArgs &a, int mode, int kp, int tpw, int prec, int gx, int gy, hipStream_t st)
{
    const int lks = loss_set(a.lu);
#define C_(P) (lks == 0 ? launch_xwide_p<P, 0>(a, mode, kp, tpw, gx, gy, st) \
                        : launch_xwide_p<P, 1>(a, mode, kp, tpw, gx, gy, st))
    GLRM_BY_PREC(prec, C_)
#undef C_
}

hipError_t launch_xwide_step(const XWideRowArgs &a, hipStream_t st)
{
    const int blocks = (int)((a.m + 15) / 16);
    hipLaunchKernelGGL(xwide_step_kernel, dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_xwide_decide(const XWideRowArgs &a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(xwide_decide_kernel, dim3(grid), dim3(XDEC_THREADS), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_reduce_dy(const ReduceArgs &a, int kp, hipStream_t st)
{
    const int blocks = (int)((a.n * (int64_t)kp + 255) / 256);
    switch (kp) {
    case 16: hipLaunchKernelGGL((reduce_dy_kernel<16>), dim3(blocks), dim3(256), 0, st, a); break;
    case 32: hipLaunchKernelGGL((reduce_dy_kernel<32>), dim3(blocks), dim3(256), 0, st, a); break;
    case 64: hipLaunchKernelGGL((reduce_dy_kernel<64>), dim3(blocks), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce_dx(const ReduceArgs &a, hipStream_t st)
{
    const int blocks = (int)((a.m * (int64_t)a.k + 255) / 256);
    hipLaunchKernelGGL(reduce_dx_kernel, dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int PPB>
static void objective64_launch(const Obj64Args &a, int grid, hipStream_t st)
{
    const int kp = a.k <= 16 ? 16 : (a.k <= 32 ? 32 : 64);
    switch (kp) {
    case 16: hipLaunchKernelGGL((objective64_kernel<16, PPB>), dim3(grid), dim3(256), 0, st, a); break;
    case 32: hipLaunchKernelGGL((objective64_kernel<32, PPB>), dim3(grid), dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((objective64_kernel<64, PPB>), dim3(grid), dim3(256), 0, st, a); break;
    }
}

static int objective64_panels_per_block(int64_t ldp) { return ldp <= 128 ? 2 : 1; }

hipError_t launch_objective64(const Obj64Args &a, int grid, hipStream_t st)
{
    if (objective64_panels_per_block(a.ldp) == 2) objective64_launch<2>(a, grid, st);
    else objective64_launch<1>(a, grid, st);
    return hipGetLastError();
}

int xstep_blocks(int kp, int tpw, int prec, bool quad)
{
    switch (prec) {
    case P_FP32: return quad ? xstep_blocks_p<P_FP32, 0>(kp, tpw) : xstep_blocks_p<P_FP32, 1>(kp, tpw);
    case P_BF16: return quad ? xstep_blocks_p<P_BF16, 0>(kp, tpw) : xstep_blocks_p<P_BF16, 1>(kp, tpw);
    case P_BF16_PLAIN:
        return quad ? xstep_blocks_p<P_BF16_PLAIN, 0>(kp, tpw) : xstep_blocks_p<P_BF16_PLAIN, 1>(kp, tpw);
    default: return 1;
    }
}

int xwide_blocks(int kp, int tpw, int prec, bool quad)
{
    switch (prec) {
    case P_FP32: return quad ? xwide_blocks_p<P_FP32, 0>(kp, tpw) : xwide_blocks_p<P_FP32, 1>(kp, tpw);
    case P_BF16: return quad ? xwide_blocks_p<P_BF16, 0>(kp, tpw) : xwide_blocks_p<P_BF16, 1>(kp, tpw);
    case P_BF16_PLAIN:
        return quad ? xwide_blocks_p<P_BF16_PLAIN, 0>(kp, tpw) : xwide_blocks_p<P_BF16_PLAIN, 1>(kp, tpw);
    default: return 1;
    }
}

int ycheck_blocks(int kp, int tpw, int prec, bool quad)
{
    switch (prec) {
    case P_FP32: return quad ? ycheck_blocks_p<P_FP32, 0>(kp, tpw) : ycheck_blocks_p<P_FP32, 1>(kp, tpw);
    case P_BF16: return quad ? ycheck_blocks_p<P_BF16, 0>(kp, tpw) : ycheck_blocks_p<P_BF16, 1>(kp, tpw);
    case P_BF16_PLAIN:
        return quad ? ycheck_blocks_p<P_BF16_PLAIN, 0>(kp, tpw) : ycheck_blocks_p<P_BF16_PLAIN, 1>(kp, tpw);
    default: return 1;
    }
}

}  // namespace glrm
