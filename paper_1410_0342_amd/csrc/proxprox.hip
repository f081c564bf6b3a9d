// The prox-prox update for quadratic losses (Sections 7.2, 7.3), dense layout.
// See proxprox.h.  Per half-step: a Gram pass over the table (the dense
// contraction: 4 x 4 register tiles of G_i per thread, the fixed factor's rows
// staged in LDS), a solve pass (one wavefront per row: Cholesky of
// G_i + I / (2 alpha) in double in LDS, then `inner` prox-prox updates by
// triangular solves), and a check pass (old and trial row objectives summed
// from the table, the step rule of Section 7.2).  Every sum has a fixed order.
#include <algorithm>

#include "glrm_kernels.h"
#include "proxprox.h"

namespace glrm {

static unsigned nblk(int64_t n, int per = 256) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

template <int KP>
constexpr int PP_NT = KP / 4;                         // 4 x 4 tiles a side
template <int KP>
constexpr int PP_UT = PP_NT<KP> * (PP_NT<KP> + 1) / 2;  // upper tiles
template <int KP>
constexpr int PP_GSZ = PP_UT<KP> * 16 + KP;           // floats of one row's Gram data

int pp_gram_floats(int kp)
{
    switch (kp) {
    case 16: return PP_GSZ<16>;
    case 32: return PP_GSZ<32>;
    default: return PP_GSZ<64>;
    }
}

// upper tile u -> (ta, tb), ta <= tb, rows of the upper triangle in order
template <int NT>
__device__ __forceinline__ void tile_of(int u, int &ta, int &tb)
{
    ta = 0;
#pragma unroll
    for (int r = 0; r < NT; ++r) {
        const int len = NT - r;
        if (u < len) {
            ta = r;
            tb = r + u;
            return;
        }
        u -= len;
    }
    ta = tb = -1;
}

// ---- Gram pass --------------------------------------------------------------------
template <int KP>
__global__ __launch_bounds__(256) void pp_gram_kernel(PPArgs a)
{
    constexpr int NT = PP_NT<KP>, UT = PP_UT<KP>, GSZ = PP_GSZ<KP>;
    constexpr int R = KP <= 32 ? 16 : 4;       // rows per workgroup
    constexpr int S = 256 / R;                 // threads per row
    constexpr int TPT = (UT + S - 1) / S;      // tiles per thread
    constexpr int CH = 64;                     // staged columns
    __shared__ float sV[CH][KP + 4];
    __shared__ float sT[R][CH + 1];
    __shared__ float sW[CH];
    const int t = threadIdx.x, r = t / S, sl = t % S;
    const int64_t i = (int64_t)blockIdx.x * R + r;
    const int64_t per = (a.cols + a.splits - 1) / a.splits;
    const int64_t c0 = (int64_t)blockIdx.y * per, c1 = min<int64_t>(a.cols, c0 + per);
    int ta[TPT], tb[TPT];
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        const int u = sl + S * q;
        if (u < UT) tile_of<NT>(u, ta[q], tb[q]);
        else ta[q] = tb[q] = -1;
    }
    float acc[TPT][16];
#pragma unroll
    for (int q = 0; q < TPT; ++q)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[q][e] = 0.0f;
    float bacc[4] = {0.f, 0.f, 0.f, 0.f};
    const float wr = (a.wrow && i < a.rows) ? a.wrow[i] : 1.0f;
    const float qnan = __builtin_nanf("");
    for (int64_t j0 = c0; j0 < c1; j0 += CH) {
        __syncthreads();
        for (int e = t; e < CH * KP; e += 256) {
            const int jj = e / KP, c = e % KP;
            const int64_t j = j0 + jj;
            sV[jj][c] = (j < c1 && c < a.k) ? a.V[j * a.k + c] : 0.0f;
        }
        for (int e = t; e < R * CH; e += 256) {
            const int rr = e / CH, jj = e % CH;
            const int64_t ii = (int64_t)blockIdx.x * R + rr, j = j0 + jj;
            sT[rr][jj] = (ii < a.rows && j < c1) ? a.T[ii * a.ldt + j] : qnan;
        }
        if (t < CH) {
            const int64_t j = j0 + t;
            sW[t] = (a.wcol && j < c1) ? a.wcol[j] : 1.0f;
        }
        __syncthreads();
        const int jn = (int)min<int64_t>(CH, c1 - j0);
        for (int jj = 0; jj < jn; ++jj) {
            const float av = sT[r][jj];
            if (av == av) {
                const float w = wr * sW[jj];
#pragma unroll
                for (int q = 0; q < TPT; ++q) {
                    if (ta[q] < 0) continue;
                    const float4 ya = *reinterpret_cast<const float4 *>(&sV[jj][4 * ta[q]]);
                    const float4 yb = *reinterpret_cast<const float4 *>(&sV[jj][4 * tb[q]]);
                    const float wa[4] = {w * ya.x, w * ya.y, w * ya.z, w * ya.w};
                    const float bb[4] = {yb.x, yb.y, yb.z, yb.w};
#pragma unroll
                    for (int p = 0; p < 4; ++p)
#pragma unroll
                        for (int qq = 0; qq < 4; ++qq) acc[q][4 * p + qq] += wa[p] * bb[qq];
                }
                if (sl < NT) {
                    const float4 y = *reinterpret_cast<const float4 *>(&sV[jj][4 * sl]);
                    const float wa = w * av;
                    bacc[0] += wa * y.x; bacc[1] += wa * y.y; bacc[2] += wa * y.z; bacc[3] += wa * y.w;
                }
            }
        }
    }
    if (i >= a.rows) return;
    float *out = a.splits > 1 ? a.gpart + ((int64_t)blockIdx.y * a.rows + i) * GSZ : a.gram + i * GSZ;
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        const int u = sl + S * q;
        if (u < UT)
#pragma unroll
            for (int e = 0; e < 16; ++e) out[u * 16 + e] = acc[q][e];
    }
    if (sl < NT)
#pragma unroll
        for (int p = 0; p < 4; ++p) out[UT * 16 + 4 * sl + p] = bacc[p];
}

__global__ void pp_reduce_kernel(const float *part, int32_t np, int64_t len, float *out)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= len) return;
    float s = 0.0f;
    for (int p = 0; p < np; ++p) s += part[(int64_t)p * len + e];
    out[e] = s;
}

template <int KP>
static hipError_t pp_gram(const PPArgs &a, hipStream_t st)
{
    constexpr int R = KP <= 32 ? 16 : 4;
    hipLaunchKernelGGL(pp_gram_kernel<KP>, dim3(nblk(a.rows, R), a.splits), dim3(256), 0, st, a);
    if (a.splits > 1) {
        const int64_t len = a.rows * (int64_t)PP_GSZ<KP>;
        hipLaunchKernelGGL(pp_reduce_kernel, dim3(nblk(len)), dim3(256), 0, st, a.gpart, a.splits, len, a.gram);
    }
    return hipGetLastError();
}

hipError_t launch_pp_gram(const PPArgs &a, hipStream_t st)
{
    switch (a.kp) {
    case 16: return pp_gram<16>(a, st);
    case 32: return pp_gram<32>(a, st);
    case 64: return pp_gram<64>(a, st);
    default: return hipErrorInvalidValue;
    }
}

// ---- solve pass: one wavefront per row ------------------------------------------
__device__ __forceinline__ double prox_elem64(const Reg &r, double alpha, double v, int c)
{
    if (c == 0 && r.offset) return r.offset == 1 ? 1.0 : v;
    switch (r.kind) {
    case R_QUAD: return v / (1.0 + 2.0 * alpha * (double)r.w);
    case R_L1: {
        const double t = fabs(v) - alpha * (double)r.w;
        return t > 0.0 ? copysign(t, v) : 0.0;
    }
    case R_NONNEG: return v > 0.0 ? v : 0.0;
    default: return v;
    }
}

template <int KP>
__global__ __launch_bounds__(64) void pp_solve_kernel(PPArgs a)
{
    constexpr int NT = PP_NT<KP>, UT = PP_UT<KP>, GSZ = PP_GSZ<KP>;
    __shared__ double sM[KP][KP + 1];
    __shared__ double sR[KP];
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    const float *g = a.gram + i * GSZ;
    const int k = a.k;
    const double al = (double)a.alpha[i];
    const double h = 1.0 / (2.0 * al);
    // the symmetric matrix from its upper tiles
    for (int e = lane; e < UT * 16; e += 64) {
        int ta, tb;
        tile_of<NT>(e >> 4, ta, tb);
        const int rr = 4 * ta + ((e >> 2) & 3), cc = 4 * tb + (e & 3);
        const double v = (double)g[e];
        sM[rr][cc] = v;
        sM[cc][rr] = v;
    }
    __syncthreads();
    // coordinates past k: identity rows (the lower part is all the factorization reads)
    if (lane < KP) {
        for (int c = 0; c <= lane; ++c)
            if (lane >= k || c >= k) sM[lane][c] = lane == c ? 1.0 : 0.0;
        if (lane < k) sM[lane][lane] += h;
    }
    __syncthreads();
    // Cholesky, lower triangle in place
    for (int j = 0; j < KP; ++j) {
        if (lane == j) {
            double d = sM[j][j];
            for (int l = 0; l < j; ++l) d -= sM[j][l] * sM[j][l];
            sM[j][j] = sqrt(d);
        }
        __syncthreads();
        if (lane > j && lane < KP) {
            double s = sM[lane][j];
            for (int l = 0; l < j; ++l) s -= sM[lane][l] * sM[j][l];
            sM[lane][j] = s / sM[j][j];
        }
        __syncthreads();
    }
    const double bc = lane < k ? (double)g[UT * 16 + lane] : 0.0;
    double x = lane < k ? (double)a.U[i * k + lane] : 0.0;
    for (int it = 0; it < a.inner; ++it) {
        if (lane < KP) sR[lane] = bc + h * x;
        __syncthreads();
        for (int j = 0; j < KP; ++j) {        // L y = rhs
            if (lane == j) sR[j] = sR[j] / sM[j][j];
            __syncthreads();
            if (lane > j && lane < KP) sR[lane] -= sM[lane][j] * sR[j];
            __syncthreads();
        }
        for (int j = KP - 1; j >= 0; --j) {   // L^T x = y
            if (lane == j) sR[j] = sR[j] / sM[j][j];
            __syncthreads();
            if (lane < j) sR[lane] -= sM[j][lane] * sR[j];
            __syncthreads();
        }
        x = lane < k ? prox_elem64(a.reg, al, sR[lane], lane) : 0.0;
        __syncthreads();
    }
    if (lane < k) a.trial[i * k + lane] = (float)x;
}

hipError_t launch_pp_solve(const PPArgs &a, hipStream_t st)
{
    if (a.rows <= 0) return hipSuccess;
    switch (a.kp) {
    case 16: hipLaunchKernelGGL(pp_solve_kernel<16>, dim3((unsigned)a.rows), dim3(64), 0, st, a); break;
    case 32: hipLaunchKernelGGL(pp_solve_kernel<32>, dim3((unsigned)a.rows), dim3(64), 0, st, a); break;
    case 64: hipLaunchKernelGGL(pp_solve_kernel<64>, dim3((unsigned)a.rows), dim3(64), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- check pass: old and trial loss sums per row (split partials), then the rule
template <int KP>
__global__ __launch_bounds__(256) void pp_check_kernel(PPArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= a.rows) return;
    const int k = a.k;
    float xo[KP], xt[KP];
#pragma unroll
    for (int c = 0; c < KP; ++c) {
        xo[c] = c < k ? a.U[i * k + c] : 0.0f;
        xt[c] = c < k ? a.trial[i * k + c] : 0.0f;
    }
    const int64_t per = (a.cols + a.splits - 1) / a.splits;
    const int64_t c0 = (int64_t)blockIdx.y * per, c1 = min<int64_t>(a.cols, c0 + per);
    const float wr = a.wrow ? a.wrow[i] : 1.0f;
    float lo = 0.0f, lt = 0.0f;
    for (int64_t j = c0 + lane; j < c1; j += 64) {
        const float av = a.T[i * a.ldt + j];
        if (av == av) {
            const float w = wr * (a.wcol ? a.wcol[j] : 1.0f);
            float z = 0.0f, zt = 0.0f;
            for (int c = 0; c < k; ++c) {
                const float v = a.V[j * k + c];
                z += xo[c] * v;
                zt += xt[c] * v;
            }
            const float d = av - z, dt = av - zt;
            lo += w * d * d;
            lt += w * dt * dt;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        lo += __shfl_xor(lo, o, 64);
        lt += __shfl_xor(lt, o, 64);
    }
    if (lane == 0) {
        float *fp = a.fpart + ((int64_t)blockIdx.y * a.rows + i) * 2;
        fp[0] = lo;
        fp[1] = lt;
    }
}

__global__ void pp_decide_kernel(PPArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.rows) return;
    const int k = a.k;
    float f = 0.0f, fp = 0.0f;
    for (int s = 0; s < a.splits; ++s) {
        f += a.fpart[((int64_t)s * a.rows + i) * 2];
        fp += a.fpart[((int64_t)s * a.rows + i) * 2 + 1];
    }
    float r0 = 0.0f, r1 = 0.0f;
    for (int c = 0; c < k; ++c) {
        r0 += reg_elem(a.reg, a.U[i * k + c], c);
        r1 += reg_elem_trial(a.reg, a.trial[i * k + c], c);
    }
    const float F0 = f + r0, F1 = fp + r1;
    const bool acc = F1 <= F0;
    if (acc)
        for (int c = 0; c < k; ++c) a.U[i * k + c] = a.trial[i * k + c];
    a.alpha[i] = acc ? a.alpha[i] * a.step_up : a.alpha[i] * a.step_down;
    a.rowobj[i] = a.obj_with_loss ? (double)(acc ? F1 : F0) : (double)(acc ? r1 : r0);
    a.rej[i] = acc ? 0 : 1;
}

hipError_t launch_pp_check(const PPArgs &a, hipStream_t st)
{
    if (a.rows <= 0) return hipSuccess;
    switch (a.kp) {
    case 16: hipLaunchKernelGGL(pp_check_kernel<16>, dim3(nblk(a.rows, 4), a.splits), dim3(256), 0, st, a); break;
    case 32: hipLaunchKernelGGL(pp_check_kernel<32>, dim3(nblk(a.rows, 4), a.splits), dim3(256), 0, st, a); break;
    case 64: hipLaunchKernelGGL(pp_check_kernel<64>, dim3(nblk(a.rows, 4), a.splits), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(pp_decide_kernel, dim3(nblk(a.rows)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// ---- transposed copy of the padded table ---------------------------------------------
__global__ __launch_bounds__(256) void transpose_kernel(const float *src, int64_t rows, int64_t cols, float *dst)
{
    __shared__ float tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int q = ty; q < 32; q += 8) {
        const int64_t r = r0 + q, c = c0 + tx;
        tile[q][tx] = (r < rows && c < cols) ? src[r * cols + c] : 0.0f;
    }
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int64_t c = c0 + q, r = r0 + tx;
        if (c < cols && r < rows) dst[c * rows + r] = tile[tx][q];
    }
}

hipError_t launch_transpose(const float *src, int64_t rows, int64_t cols, float *dst, hipStream_t st)
{
    hipLaunchKernelGGL(transpose_kernel, dim3(nblk(cols, 32), nblk(rows, 32)), dim3(256), 0, st, src, rows, cols, dst);
    return hipGetLastError();
}

// ---- the sweep's objective: decided column objectives + r of the decided rows ----
__global__ __launch_bounds__(256) void pp_finalize_kernel(const double *rx, const int32_t *jx, int64_t m,
                                                          const double *ry, const int32_t *jy, int64_t n,
                                                          double *stats, long long *istats, double *history,
                                                          int32_t sweep)
{
    __shared__ double sF[256];
    __shared__ long long sa[256], sb[256];
    double F = 0.0;
    long long ra = 0, rb = 0;
    for (int64_t q = threadIdx.x; q < n; q += 256) { F += ry[q]; rb += jy[q]; }
    for (int64_t q = threadIdx.x; q < m; q += 256) { F += rx[q]; ra += jx[q]; }
    sF[threadIdx.x] = F;
    sa[threadIdx.x] = ra;
    sb[threadIdx.x] = rb;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sF[threadIdx.x] += sF[threadIdx.x + o];
            sa[threadIdx.x] += sa[threadIdx.x + o];
            sb[threadIdx.x] += sb[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        stats[0] = sF[0];
        istats[0] = sa[0];
        istats[1] = sb[0];
        if (history) history[sweep] = sF[0];
    }
}

hipError_t launch_pp_finalize(const double *rowobj_x, const int32_t *rej_x, int64_t m, const double *rowobj_y,
                              const int32_t *rej_y, int64_t n, double *part, double *stats, long long *istats,
                              double *history, int32_t sweep, hipStream_t st)
{
    (void)part;
    hipLaunchKernelGGL(pp_finalize_kernel, dim3(1), dim3(256), 0, st, rowobj_x, rej_x, m, rowobj_y, rej_y, n, stats,
                       istats, history, sweep);
    return hipGetLastError();
}

}  // namespace glrm
