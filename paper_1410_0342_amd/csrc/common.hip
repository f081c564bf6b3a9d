// Set-up and element-wise kernels: packing the dense table, observation
// counts and initial step sizes (Section 7.2: alpha^0 = scale / n_i), the prox
// of a regularizer over the rows of a factor, regularizer sums, and fixed-order
// double reductions.
#include "glrm_device.h"
#include "glrm_kernels.h"

namespace glrm {

// Packed column j of row i: whether it is observed, and its value.
__device__ __forceinline__ bool pack_entry(const PackArgs &a, int64_t i, int64_t j, float &v)
{
    const int64_t s = a.emb.src ? a.emb.src[j] : j;
    if (a.mask && a.mask[i * a.lda + s] == 0) return false;
    const float x = a.A[i * a.lda + s];
    if (!a.emb.src || a.emb.kind[j] == EMB_COPY) v = x;
    else if (a.emb.kind[j] == EMB_EQ) v = x == (float)a.emb.thr[j] ? 1.0f : -1.0f;
    else v = x > (float)a.emb.thr[j] ? 1.0f : -1.0f;
    return true;
}

// One workgroup per 16 rows of the padded table.  Unobserved and padding
// entries become quiet NaN.  Row counts are exact block sums; column counts
// are integer atomics (order-free, so deterministic).
__global__ __launch_bounds__(256) void pack_dense_kernel(PackArgs a)
{
    __shared__ int s_cnt[4];
    const int64_t i0 = (int64_t)blockIdx.x * 16;
    const float qnan = __builtin_nanf("");
    for (int ii = 0; ii < 16; ++ii) {
        const int64_t i = i0 + ii;
        int cnt = 0;
        for (int64_t j = threadIdx.x; j < a.ldp; j += 256) {
            float v = qnan;
            if (i < a.m && j < a.n && pack_entry(a, i, j, v)) ++cnt;
            a.Ap[i * a.ldp + j] = v;
        }
        cnt = (int)sum_lanes<64>((float)cnt);
        if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = cnt;
        __syncthreads();
        if (threadIdx.x == 0 && i < a.m) a.row_count[i] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        __syncthreads();
    }
    for (int64_t j = threadIdx.x; j < a.n; j += 256) {
        int cnt = 0;
        for (int ii = 0; ii < 16; ++ii) {
            const int64_t i = i0 + ii;
            if (i < a.m) cnt += a.mask ? (a.mask[i * a.lda + (a.emb.src ? a.emb.src[j] : j)] != 0) : 1;
        }
        if (cnt) atomicAdd(&a.col_count[j], cnt);
    }
}

hipError_t launch_pack_dense(const PackArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(pack_dense_kernel, dim3((unsigned)(a.mp / 16)), dim3(256), 0, st, a);
    return hipGetLastError();
}

__global__ void init_alpha_kernel(const int32_t *count, int64_t len, float scale, float *alpha)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < len) {
        const int c = count[t];
        alpha[t] = scale / (float)(c > 0 ? c : 1);
    }
}

hipError_t launch_init_alpha(const int32_t *count, int64_t len, float scale, float *alpha, hipStream_t st)
{
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL(init_alpha_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, count, len, scale,
                       alpha);
    return hipGetLastError();
}

__global__ void prox_kernel(Reg r, float *V, int64_t rows, int32_t k, int64_t ldv, const float *alpha)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= rows * k) return;
    const int64_t i = t / k;
    const int c = (int)(t % k);
    const float al = alpha ? alpha[i] : 1.0f;
    V[i * ldv + c] = prox_elem(r, al, V[i * ldv + c], c);
}

hipError_t launch_prox(Reg r, float *V, int64_t rows, int32_t k, int64_t ldv, const float *alpha, hipStream_t st)
{
    const int64_t total = rows * k;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(prox_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, r, V, rows, k, ldv,
                       alpha);
    return hipGetLastError();
}

// dV += the regularizer's least-magnitude subgradient at V, element-wise.
__global__ void reg_grad_kernel(Reg r, const float *V, int64_t rows, int32_t k, float *dV)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= rows * k) return;
    dV[t] += reg_grad_elem(r, V[t], (int)(t % k));
}

hipError_t launch_reg_grad(Reg r, const float *V, int64_t rows, int32_t k, float *dV, hipStream_t st)
{
    const int64_t total = rows * k;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(reg_grad_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, r, V, rows, k, dV);
    return hipGetLastError();
}

// Regularizer sum over a factor, in double; one partial per workgroup.  A
// thread's coordinate advances with its flat index (one division per thread,
// then a compare and subtract per step).
__global__ __launch_bounds__(256) void regsum_kernel(Reg r, const float *V, int64_t rows, int32_t k, double *part)
{
    __shared__ double s[4];
    double acc = 0.0;
    const int64_t total = rows * k, stride = (int64_t)gridDim.x * 256;
    const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int dc = (int)(stride % k);
    int c = (int)(t0 % k);
    for (int64_t t = t0; t < total; t += stride) {
        acc += reg_elem64(r, (double)V[t], c);
        c += dc;
        if (c >= k) c -= k;
    }
    acc = sum_lanes64<64>(acc);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

hipError_t launch_regsum(Reg r, const float *V, int64_t rows, int32_t k, double *part, int blocks, hipStream_t st)
{
    hipLaunchKernelGGL(regsum_kernel, dim3(blocks), dim3(256), 0, st, r, V, rows, k, part);
    return hipGetLastError();
}

// out = sum(a) + sum(b), fixed order (one workgroup, tree in LDS).
__global__ __launch_bounds__(256) void sum_doubles_kernel(const double *a, int32_t na, const double *b, int32_t nb,
                                                          double *out)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int q = threadIdx.x; q < na; q += 256) acc += a[q];
    for (int q = threadIdx.x; q < nb; q += 256) acc += b[q];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

hipError_t launch_sum_doubles(const double *a, int32_t na, const double *b, int32_t nb, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(sum_doubles_kernel, dim3(1), dim3(256), 0, st, a, na, b, nb, out);
    return hipGetLastError();
}

// dst[j] = src[map[j]] (src[j] without a map; 1 without src) for j < n, 1 for
// the padding columns up to ldp.
__global__ void pad_weights_kernel(const float *src, const int32_t *map, int64_t n, int64_t ldp, float *dst)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < ldp) dst[j] = (src && j < n) ? src[map ? map[j] : j] : 1.0f;
}

hipError_t launch_pad_weights(const float *src, const int32_t *map, int64_t n, int64_t ldp, float *dst,
                              hipStream_t st)
{
    hipLaunchKernelGGL(pad_weights_kernel, dim3((unsigned)((ldp + 255) / 256)), dim3(256), 0, st, src, map, n, ldp,
                       dst);
    return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t *p, int64_t len, int32_t v)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < len) p[t] = v;
}

hipError_t launch_fill_i32(int32_t *p, int64_t len, int32_t v, hipStream_t st)
{
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, p, len, v);
    return hipGetLastError();
}

}  // namespace glrm
