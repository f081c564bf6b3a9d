// Kernels of the linear algebra around the fit (declared in linalg.h): the
// matrices defined entry by entry on the observed set, their products with
// blocks of vectors, tall-skinny products with the factors, and vector
// reductions.  Everything is summed in double and in a fixed order, so each
// result is reproducible.  None of this is on the sweep's hot path: these
// serve the certificate of Section 7.6 (a few hundred matrix-vector pairs)
// and the randomized SVD of Section 7.5 (a few block products).
#include <algorithm>

#include "glrm_kernels.h"
#include "linalg.h"

namespace glrm {

static unsigned nblk(int64_t n, int per = 256) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

// ---- entry-wise matrices -------------------------------------------------------

// One workgroup per padded table row; x_i staged in LDS, z = x_i . y_j and the
// derivative in double (the branch at a kink is taken on the double product).
__global__ __launch_bounds__(256) void dense_grad_matrix_kernel(EntryArgs a, float *V)
{
    __shared__ float sx[GLRM_MAXK_DEV];
    const int64_t i = blockIdx.x;
    if (threadIdx.x < a.k) sx[threadIdx.x] = i < a.m ? a.X[i * a.k + threadIdx.x] : 0.0f;
    __syncthreads();
    for (int64_t j = threadIdx.x; j < a.ldp; j += 256) {
        float out = 0.0f;
        const float av = a.Ap[i * a.ldp + j];
        if (i < a.m && j < a.n && av == av) {
            double z = 0.0;
            for (int l = 0; l < a.k; ++l) z += (double)sx[l] * (double)a.Y[j * a.k + l];
            const int q = a.lt.uniform >= 0 ? a.lt.uniform : a.codes[j];
            const double gv = loss_g64(a.lt.kind[q], a.lt.levels[q], (double)a.lt.param[q], z, (double)av);
            out = (float)(a.colw ? gv * (double)a.colw[j] : gv);
        }
        V[i * a.ldp + j] = out;
    }
}

hipError_t launch_dense_grad_matrix(const EntryArgs &a, float *V, hipStream_t st)
{
    hipLaunchKernelGGL(dense_grad_matrix_kernel, dim3((unsigned)a.mp), dim3(256), 0, st, a, V);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void dense_scaled_matrix_kernel(EntryArgs a, float *V)
{
    const int64_t i = blockIdx.x;
    for (int64_t j = threadIdx.x; j < a.ldp; j += 256) {
        const float av = a.Ap[i * a.ldp + j];
        V[i * a.ldp + j] = (i < a.m && j < a.n && av == av) ? a.cs[j] * (av - a.mu[j]) : 0.0f;
    }
}

hipError_t launch_dense_scaled_matrix(const EntryArgs &a, float *V, hipStream_t st)
{
    hipLaunchKernelGGL(dense_scaled_matrix_kernel, dim3((unsigned)a.mp), dim3(256), 0, st, a, V);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void coo_grad_values_kernel(EntryArgs a, const int32_t *row, const int32_t *col,
                                                              const float *A, int64_t nnz, float *out)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nnz) return;
    const int64_t i = row[e], j = col[e];
    double z = 0.0;
    if ((a.k & 3) == 0 && (((uintptr_t)a.X | (uintptr_t)a.Y) & 15) == 0) {
        // factors on 16 bytes with rows of a multiple of four floats: four
        // coordinates per load, summed in the same order
        const float4 *x4 = reinterpret_cast<const float4 *>(a.X + i * a.k);
        const float4 *y4 = reinterpret_cast<const float4 *>(a.Y + j * a.k);
        for (int l = 0; l < a.k / 4; ++l) {
            const float4 xv = x4[l], yv = y4[l];
            z += (double)xv.x * (double)yv.x;
            z += (double)xv.y * (double)yv.y;
            z += (double)xv.z * (double)yv.z;
            z += (double)xv.w * (double)yv.w;
        }
    } else {
        for (int l = 0; l < a.k; ++l) z += (double)a.X[i * a.k + l] * (double)a.Y[j * a.k + l];
    }
    const int q = a.lt.uniform >= 0 ? a.lt.uniform : a.codes[j];
    const double gv = loss_g64(a.lt.kind[q], a.lt.levels[q], (double)a.lt.param[q], z, (double)A[e]);
    out[e] = (float)(a.colw ? gv * (double)a.colw[j] : gv);
}

hipError_t launch_coo_grad_values(const EntryArgs &a, const int32_t *row, const int32_t *col, const float *A,
                                  int64_t nnz, float *out, hipStream_t st)
{
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(coo_grad_values_kernel, dim3(nblk(nnz)), dim3(256), 0, st, a, row, col, A, nnz, out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void coo_scaled_values_kernel(EntryArgs a, const int32_t *col, const float *A,
                                                                int64_t nnz, float *out)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nnz) return;
    const int64_t j = col[e];
    out[e] = a.cs[j] * (A[e] - a.mu[j]);
}

hipError_t launch_coo_scaled_values(const EntryArgs &a, const int32_t *col, const float *A, int64_t nnz, float *out,
                                    hipStream_t st)
{
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(coo_scaled_values_kernel, dim3(nblk(nnz)), dim3(256), 0, st, a, col, A, nnz, out);
    return hipGetLastError();
}

__global__ void permute_kernel(const int32_t *perm, const float *in, int64_t nnz, float *out)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < nnz) out[p] = in[perm[p]];
}

hipError_t launch_permute(const int32_t *perm, const float *in, int64_t nnz, float *out, hipStream_t st)
{
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(permute_kernel, dim3(nblk(nnz)), dim3(256), 0, st, perm, in, nnz, out);
    return hipGetLastError();
}

// ---- the table's matrix times a block of vectors -----------------------------------

// Blocks of vectors go through the matrix cores in double: v_mfma_f64_16x16x4f64
// adds A (16 x 4) B (4 x 16) to a 16 x 16 accumulator.  Lane l supplies
// A[l & 15][l >> 4] and B[l >> 4][l & 15] and holds D[(l >> 4) + 4 v][l & 15]
// in element v of the accumulator (rows interleaved by four, unlike the fp32
// 16 x 16 x 4 product's consecutive rows).  The table's floats convert to double
// exactly, so a product differs from the plain double sum in its order only.
typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 mfma64(double a, double b, dbl4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int LA_NT = (LA_MAXB + 15) / 16;   // 16-wide tiles of the widest block

// out (m x b) = alpha V B.  A wavefront owns R tiles of 16 rows and every
// 16-wide tile of the block (NT of them).  The table's columns are the
// contraction, 16 per step: lane (i, q) loads four consecutive floats of row
// i, and the step's product s contracts column 4 q + s, with the rows of B
// loaded to match.  The accumulators pass through LDS on their way out, so no
// branch separates the last product from the first read of its result.
template <int NT, int R>
__global__ __launch_bounds__(256) void dense_apply_kernel(const float *V, int64_t m, int64_t n, int64_t ldp,
                                                          const double *B, int32_t b, double alpha, double *out)
{
    __shared__ double sOut[4][R * NT][256];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), li = lane & 15, lq = lane >> 4;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + w) * (16 * R);
    dbl4 acc[R][NT];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[r][t] = dbl4{0.0, 0.0, 0.0, 0.0};
    if (row0 < m) {
#pragma unroll 2
        for (int64_t j0 = 0; j0 < n; j0 += 16) {
            const int64_t j = j0 + 4 * lq;
            double bf[NT][4];
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int c = 16 * t + li;
                    bf[t][s] = (j + s < n && c < b) ? B[(j + s) * b + c] : 0.0;
                }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t i = row0 + 16 * r + li;
                float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                // j0 + 16 <= ldp (a multiple of 16), so the four floats lie in the row
                if (i < m) v = *reinterpret_cast<const float4 *>(V + i * ldp + j);
                const double vs[4] = {j < n ? (double)v.x : 0.0, j + 1 < n ? (double)v.y : 0.0,
                                      j + 2 < n ? (double)v.z : 0.0, j + 3 < n ? (double)v.w : 0.0};
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int s = 0; s < 4; ++s) acc[r][t] = mfma64(vs[s], bf[t][s], acc[r][t]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            acc[r][t] = mfma64(0.0, 0.0, acc[r][t]);   // in order behind the last product
#pragma unroll
            for (int v = 0; v < 4; ++v) sOut[w][r * NT + t][64 * v + lane] = acc[r][t][v];
        }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = row0 + 16 * r + lq + 4 * v;
                const int c = 16 * t + li;
                if (i < m && c < b) out[i * b + c] = alpha * sOut[w][r * NT + t][64 * v + lane];
            }
}

template <int NT>
static void apply_launch(const float *V, int64_t m, int64_t n, int64_t ldp, const double *B, int32_t b, double alpha,
                         double *out, hipStream_t st)
{
    constexpr int R = NT <= 2 ? 2 : 1;
    hipLaunchKernelGGL((dense_apply_kernel<NT, R>), dim3(nblk(m, 64 * R)), dim3(256), 0, st, V, m, n, ldp, B, b,
                       alpha, out);
}

// One vector (b = 1): out_i = alpha sum_j V_ij x_j.  A wavefront takes
// GEMV_R rows at once and lane l four consecutive columns of every 256
// (16-byte loads), so each load of x serves GEMV_R rows; the lanes' sums are
// combined by a butterfly.
constexpr int GEMV_R = 4;

__global__ __launch_bounds__(256) void dense_gemv_kernel(const float *V, int64_t m, int64_t n, int64_t ldp,
                                                         const double *x, double alpha, double *out)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t i0 = ((int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * GEMV_R; i0 < m; i0 += nw * GEMV_R) {
        double acc[GEMV_R];
#pragma unroll
        for (int r = 0; r < GEMV_R; ++r) acc[r] = 0.0;
        // j < n <= ldp, and ldp is a multiple of 16: the four floats lie in the row
        for (int64_t j = 4 * lane; j < n; j += 256) {
            const double x0 = x[j], x1 = j + 1 < n ? x[j + 1] : 0.0, x2 = j + 2 < n ? x[j + 2] : 0.0,
                         x3 = j + 3 < n ? x[j + 3] : 0.0;
#pragma unroll
            for (int r = 0; r < GEMV_R; ++r) {
                // rows past the last re-read it; their sums are not stored
                const int64_t i = min<int64_t>(i0 + r, m - 1);
                const float4 v = *reinterpret_cast<const float4 *>(V + i * ldp + j);
                acc[r] += (double)v.x * x0;
                acc[r] += j + 1 < n ? (double)v.y * x1 : 0.0;
                acc[r] += j + 2 < n ? (double)v.z * x2 : 0.0;
                acc[r] += j + 3 < n ? (double)v.w * x3 : 0.0;
            }
        }
#pragma unroll
        for (int r = 0; r < GEMV_R; ++r) {
            double t = acc[r];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o, 64);
            if (lane == 0 && i0 + r < m) out[i0 + r] = alpha * t;
        }
    }
}

hipError_t launch_dense_apply(const float *V, int64_t m, int64_t n, int64_t ldp, const double *B, int32_t b,
                              double alpha, double *out, hipStream_t st)
{
    if (b < 1 || b > LA_MAXB || ldp % 16 != 0 || ldp < n) return hipErrorInvalidValue;
    if (m <= 0) return hipSuccess;
    if (b == 1) {
        const int64_t blocks = std::min<int64_t>((m + 4 * GEMV_R - 1) / (4 * GEMV_R), 8192);
        hipLaunchKernelGGL(dense_gemv_kernel, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, st, V, m, n,
                           ldp, B, alpha, out);
        return hipGetLastError();
    }
    switch ((b + 15) / 16) {
    case 1: apply_launch<1>(V, m, n, ldp, B, b, alpha, out, st); break;
    case 2: apply_launch<2>(V, m, n, ldp, B, b, alpha, out, st); break;
    case 3: apply_launch<3>(V, m, n, ldp, B, b, alpha, out, st); break;
    case 4: apply_launch<4>(V, m, n, ldp, B, b, alpha, out, st); break;
    case 5: apply_launch<5>(V, m, n, ldp, B, b, alpha, out, st); break;
    default: apply_launch<LA_NT>(V, m, n, ldp, B, b, alpha, out, st); break;
    }
    return hipGetLastError();
}

// Partials of U^T B, for U (rows x P, leading dimension ldu) and B (rows x b,
// leading dimension ldb): workgroup (x, y) takes the 16 columns 16 x of U and
// row chunk y, and writes part[y][p][c] for its p and every c < b.  The
// chunk's rows are the contraction: its four wavefronts take four consecutive
// runs of them, four rows per product, and their sums are added in wavefront
// order through LDS.
template <typename TU, typename TB, int NT>
__global__ __launch_bounds__(256) void tmul_kernel(const TU *U, int64_t rows, int64_t P, int64_t ldu, const TB *B,
                                                   int64_t ldb, int32_t b, int64_t per, double *part)
{
    __shared__ double sAcc[4][NT][256];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), li = lane & 15, lk = lane >> 4;
    const int64_t p0 = (int64_t)blockIdx.x * 16;
    const int64_t c0 = (int64_t)blockIdx.y * per, c1 = min<int64_t>(rows, c0 + per);
    const int64_t run = (max<int64_t>(c1 - c0, 0) + 3) / 4;
    const int64_t r0 = min<int64_t>(c1, c0 + w * run), r1 = min<int64_t>(c1, r0 + run);
    const bool pin = p0 + li < P;
    dbl4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int64_t i0 = r0; i0 < r1; i0 += 4) {
        const int64_t i = i0 + lk;
        const bool in = i < r1;
        const double a = (in && pin) ? (double)U[i * ldu + p0 + li] : 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = 16 * t + li;
            const double bv = (in && c < b) ? (double)B[i * ldb + c] : 0.0;
            acc[t] = mfma64(a, bv, acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        acc[t] = mfma64(0.0, 0.0, acc[t]);   // in order behind the last product
#pragma unroll
        for (int v = 0; v < 4; ++v) sAcc[w][t][64 * v + lane] = acc[t][v];
    }
    __syncthreads();
    const int e = threadIdx.x, v = e >> 6, l2 = e & 63;
    const int64_t p = p0 + (l2 >> 4) + 4 * v;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = 16 * t + (l2 & 15);
        if (p < P && c < b)
            part[((int64_t)blockIdx.y * P + p) * b + c] =
                ((sAcc[0][t][e] + sAcc[1][t][e]) + sAcc[2][t][e]) + sAcc[3][t][e];
    }
}

template <typename TU, typename TB>
static hipError_t tmul_launch(const TU *U, int64_t rows, int64_t P, int64_t ldu, const TB *B, int64_t ldb, int32_t b,
                              int chunks, double *part, hipStream_t st)
{
    if (b < 1 || b > LA_MAXB) return hipErrorInvalidValue;
    const int64_t per = (rows + chunks - 1) / chunks;
    const dim3 grid((unsigned)((P + 15) / 16), (unsigned)chunks);
    switch ((b + 15) / 16) {
    case 1: hipLaunchKernelGGL((tmul_kernel<TU, TB, 1>), grid, dim3(256), 0, st, U, rows, P, ldu, B, ldb, b, per, part); break;
    case 2: hipLaunchKernelGGL((tmul_kernel<TU, TB, 2>), grid, dim3(256), 0, st, U, rows, P, ldu, B, ldb, b, per, part); break;
    case 3: hipLaunchKernelGGL((tmul_kernel<TU, TB, 3>), grid, dim3(256), 0, st, U, rows, P, ldu, B, ldb, b, per, part); break;
    case 4: hipLaunchKernelGGL((tmul_kernel<TU, TB, 4>), grid, dim3(256), 0, st, U, rows, P, ldu, B, ldb, b, per, part); break;
    case 5: hipLaunchKernelGGL((tmul_kernel<TU, TB, 5>), grid, dim3(256), 0, st, U, rows, P, ldu, B, ldb, b, per, part); break;
    default: hipLaunchKernelGGL((tmul_kernel<TU, TB, LA_NT>), grid, dim3(256), 0, st, U, rows, P, ldu, B, ldb, b, per, part); break;
    }
    return hipGetLastError();
}

// out[e] = alpha * sum over p of part[p][e].  A workgroup takes 64 consecutive
// e; wavefront w sums the partials p = w, w + 4, ... in order, and the four
// sums are added in wavefront order.
__global__ __launch_bounds__(256) void reduce_parts_kernel(const double *part, int32_t np, int64_t len, double alpha,
                                                           double *out)
{
    __shared__ double s[4][64];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // scalar: loops over w stay uniform
    const int64_t e = (int64_t)blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (e < len) {
        // loads run ahead; the sum keeps the order of p
#pragma unroll 8
        for (int p = w; p < np; p += 4) acc += part[(int64_t)p * len + e];
    }
    s[w][lane] = acc;
    __syncthreads();
    if (w == 0 && e < len) out[e] = alpha * (((s[0][lane] + s[1][lane]) + s[2][lane]) + s[3][lane]);
}

static void reduce_parts(const double *part, int32_t np, int64_t len, double alpha, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(nblk(len, 64)), dim3(256), 0, st, part, np, len, alpha, out);
}

int dense_apply_t_chunks(int64_t m, int64_t n)
{
    const int64_t cblocks = (n + 15) / 16;
    const int64_t want = std::max<int64_t>(1, 2048 / cblocks);
    return (int)std::min<int64_t>({want, (int64_t)LA_TCHUNKS, std::max<int64_t>(1, (m + 63) / 64)});
}

// One vector (b = 1): partials of V^T q per row chunk.  A workgroup takes 256
// columns (lane -> four consecutive columns, 16-byte loads) and a chunk of
// rows, its four wavefronts every fourth row; the four sums are combined in
// order.
__global__ __launch_bounds__(256) void dense_gemv_t_kernel(const float *V, int64_t m, int64_t n, int64_t ldp,
                                                           const double *q, int64_t per, double *part)
{
    __shared__ double sAcc[4][256];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // scalar: loops over w stay uniform
    const int64_t j = ((int64_t)blockIdx.x * 64 + lane) * 4;
    const int64_t r0 = (int64_t)blockIdx.y * per, r1 = min<int64_t>(m, r0 + per);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    // j < n <= ldp, and ldp is a multiple of 16: the four floats lie in the row
    if (j < n) {
#pragma unroll 4
        for (int64_t i = r0 + w; i < r1; i += 4) {
            const float4 v = *reinterpret_cast<const float4 *>(V + i * ldp + j);
            const double qi = q[i];
            a0 += (double)v.x * qi;
            a1 += (double)v.y * qi;
            a2 += (double)v.z * qi;
            a3 += (double)v.w * qi;
        }
    }
    sAcc[w][4 * lane] = a0;
    sAcc[w][4 * lane + 1] = a1;
    sAcc[w][4 * lane + 2] = a2;
    sAcc[w][4 * lane + 3] = a3;
    __syncthreads();
    const int t = threadIdx.x;
    const int64_t jj = (int64_t)blockIdx.x * 256 + t;
    if (jj < n) part[(int64_t)blockIdx.y * n + jj] = ((sAcc[0][t] + sAcc[1][t]) + sAcc[2][t]) + sAcc[3][t];
}

hipError_t launch_dense_apply_t(const float *V, int64_t m, int64_t n, int64_t ldp, const double *Q, int32_t b,
                                double alpha, double *part, double *out, hipStream_t st)
{
    if (b < 1 || b > LA_MAXB || ldp % 16 != 0 || ldp < n) return hipErrorInvalidValue;
    if (n <= 0) return hipSuccess;
    if (b == 1) {
        // row chunks: enough workgroups to fill the device, partials within LA_TCHUNKS n
        const int64_t cblocks = (n + 255) / 256;
        const int ch = (int)std::min<int64_t>({(int64_t)LA_TCHUNKS, std::max<int64_t>(1, 4096 / cblocks),
                                               std::max<int64_t>(1, (m + 255) / 256)});
        const int64_t per = (m + ch - 1) / ch;
        hipLaunchKernelGGL(dense_gemv_t_kernel, dim3((unsigned)cblocks, ch), dim3(256), 0, st, V, m, n, ldp, Q, per,
                           part);
        reduce_parts(part, ch, n, alpha, out, st);
        return hipGetLastError();
    }
    const int ch = dense_apply_t_chunks(m, n);
    hipError_t e = tmul_launch<float, double>(V, m, n, ldp, Q, b, b, ch, part, st);
    if (e != hipSuccess) return e;
    reduce_parts(part, ch, n * b, alpha, out, st);
    return hipGetLastError();
}

// One wavefront per segment (row of the row view, or column of the column
// view).  Narrow blocks: lanes take every 64th entry and the lanes' sums are
// combined by a butterfly; wide blocks: lanes take output columns.
__global__ __launch_bounds__(256) void seg_apply_kernel(const int32_t *ptr, const int32_t *idx, const float *val,
                                                        int64_t rows, const double *B, int32_t b, double alpha,
                                                        double *out)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (r >= rows) return;
    const int32_t beg = ptr[r], end = ptr[r + 1];
    if (b <= 4) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int32_t e = beg + lane; e < end; e += 64) {
            const double v = (double)val[e];
            const int64_t j = idx[e];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < b) acc[c] += v * B[j * b + c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double s = acc[c];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
            if (c < b && lane == 0) out[r * b + c] = alpha * s;
        }
    } else {
        for (int c0 = 0; c0 < b; c0 += 64) {
            const int c = c0 + lane;
            double acc = 0.0;
            for (int32_t e = beg; e < end; ++e)
                if (c < b) acc += (double)val[e] * B[(int64_t)idx[e] * b + c];
            if (c < b) out[r * b + c] = alpha * acc;
        }
    }
}

hipError_t launch_seg_apply(const int32_t *ptr, const int32_t *idx, const float *val, int64_t rows, const double *B,
                            int32_t b, double alpha, double *out, hipStream_t st)
{
    if (b < 1 || b > LA_MAXB) return hipErrorInvalidValue;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(seg_apply_kernel, dim3(nblk(rows, 4)), dim3(256), 0, st, ptr, idx, val, rows, B, b, alpha,
                       out);
    return hipGetLastError();
}

// ---- tall-skinny products ----------------------------------------------------------

constexpr int TALL_ROWS = 256;       // rows per workgroup of U^T B, at least
constexpr int TALL_CHUNKS = 1024;    // workgroups along the rows, at most

int tall_tmul_blocks(int64_t rows)
{
    return (int)std::min<int64_t>(TALL_CHUNKS, std::max<int64_t>(1, (rows + TALL_ROWS - 1) / TALL_ROWS));
}

template <typename TU, typename TB>
static hipError_t tall_tmul(const TU *U, int64_t rows, int32_t k, int64_t ldu, const TB *B, int64_t ldb, int32_t b,
                            double *part, double *out, hipStream_t st)
{
    if (k < 1 || b < 1 || b > LA_MAXB) return hipErrorInvalidValue;
    const int nb = tall_tmul_blocks(rows);
    hipError_t e = tmul_launch<TU, TB>(U, rows, k, ldu, B, ldb, b, nb, part, st);
    if (e != hipSuccess) return e;
    reduce_parts(part, nb, (int64_t)k * b, 1.0, out, st);
    return hipGetLastError();
}

hipError_t launch_tall_tmul_f(const float *U, int64_t rows, int32_t k, int64_t ldu, const double *B, int32_t b,
                              double *part, double *out, hipStream_t st)
{
    return tall_tmul<float, double>(U, rows, k, ldu, B, b, b, part, out, st);
}

hipError_t launch_tall_tmul_d(const double *U, int64_t rows, int32_t k, int64_t ldu, const double *B, int32_t b,
                              double *part, double *out, hipStream_t st)
{
    return tall_tmul<double, double>(U, rows, k, ldu, B, b, b, part, out, st);
}

hipError_t launch_gram_f(const float *U, int64_t rows, int32_t k, double *part, double *out, hipStream_t st)
{
    return tall_tmul<float, float>(U, rows, k, k, U, k, k, part, out, st);
}

template <typename TU>
__global__ void tall_mul_kernel(const TU *U, int64_t rows, int32_t k, int64_t ldu, const double *S, int32_t b,
                                double alpha, double beta, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= rows * b) return;
    const int64_t i = t / b;
    const int c = (int)(t % b);
    double acc = 0.0;
    for (int l = 0; l < k; ++l) acc += (double)U[i * ldu + l] * S[l * b + c];
    out[t] = (beta == 0.0 ? 0.0 : beta * out[t]) + alpha * acc;
}

hipError_t launch_tall_mul_f(const float *U, int64_t rows, int32_t k, int64_t ldu, const double *S, int32_t b,
                             double alpha, double beta, double *out, hipStream_t st)
{
    if (rows * b <= 0) return hipSuccess;
    hipLaunchKernelGGL(tall_mul_kernel<float>, dim3(nblk(rows * b)), dim3(256), 0, st, U, rows, k, ldu, S, b, alpha,
                       beta, out);
    return hipGetLastError();
}

hipError_t launch_tall_mul_d(const double *U, int64_t rows, int32_t k, int64_t ldu, const double *S, int32_t b,
                             double alpha, double beta, double *out, hipStream_t st)
{
    if (rows * b <= 0) return hipSuccess;
    hipLaunchKernelGGL(tall_mul_kernel<double>, dim3(nblk(rows * b)), dim3(256), 0, st, U, rows, k, ldu, S, b, alpha,
                       beta, out);
    return hipGetLastError();
}

// ---- vectors -------------------------------------------------------------------------

constexpr int SUMSQ_BLOCKS = 256;

__global__ __launch_bounds__(256) void sumsq_kernel(const double *v, int64_t len, double *part)
{
    __shared__ double s[4];
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256)
        acc += v[t] * v[t];
    acc = sum_lanes64<64>(acc);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

hipError_t launch_sumsq(const double *v, int64_t len, double *part, double *nrm2, hipStream_t st)
{
    hipLaunchKernelGGL(sumsq_kernel, dim3(SUMSQ_BLOCKS), dim3(256), 0, st, v, len, part);
    reduce_parts(part, SUMSQ_BLOCKS, 1, 1.0, nrm2, st);
    return hipGetLastError();
}

__global__ void normalize_kernel(double *v, int64_t len, const double *nrm2, double *est, int32_t slot)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double nv = sqrt(*nrm2);
    if (t == 0 && est) est[slot] = nv;
    if (v && t < len && nv > 0.0) v[t] /= nv;
}

hipError_t launch_normalize(double *v, int64_t len, const double *nrm2, double *est, int32_t slot, hipStream_t st)
{
    hipLaunchKernelGGL(normalize_kernel, dim3(nblk(std::max<int64_t>(len, 1))), dim3(256), 0, st, v, len, nrm2, est,
                       slot);
    return hipGetLastError();
}

__global__ void start_vector_kernel(double *v, int64_t len, uint64_t seed)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= len) return;
    // SplitMix64 (Steele, Lea, Flood 2014) of the counter seed + t
    uint64_t z = seed + (uint64_t)t * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    v[t] = 1.0 + (double)(z >> 11) * 0x1.0p-53;
}

hipError_t launch_start_vector(double *v, int64_t len, uint64_t seed, hipStream_t st)
{
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL(start_vector_kernel, dim3(nblk(len)), dim3(256), 0, st, v, len, seed);
    return hipGetLastError();
}

__global__ void to_float_kernel(const double *src, int64_t rows, int32_t b, int32_t cols, float *dst, int64_t ldd,
                                int32_t col0)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= rows * cols) return;
    const int64_t i = t / cols;
    const int c = (int)(t % cols);
    dst[i * ldd + col0 + c] = (float)src[i * b + c];
}

hipError_t launch_to_float(const double *src, int64_t rows, int32_t b, int32_t cols, float *dst, int64_t ldd,
                           int32_t col0, hipStream_t st)
{
    if (rows * cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_float_kernel, dim3(nblk(rows * cols)), dim3(256), 0, st, src, rows, b, cols, dst, ldd, col0);
    return hipGetLastError();
}

// ---- per-column sums (loss scaling) ------------------------------------------------
// Mode 0: each column's least and largest value; mode 1: the derivative sums
// at the COL_PTS points lo + (hi - lo) p / (COL_PTS + 1), p = 1..COL_PTS, of
// the column's bracket; mode 2: the loss sum at mid.  Partial sums per row
// chunk, COL_SLOTS of them per column, combined in chunk order.

// Row chunks of the dense column passes: a thread per column and chunk walks
// the chunk's rows, so a narrow table needs many chunks to fill the device.
// The chunks make at most 1024 workgroups in all, the number resident at once
// (four per CU on 256 CUs at this kernel's registers): one more would run
// alone in a second round.  Within the partials' budget.
int col_pass_chunks(int64_t m, int64_t n)
{
    const int64_t cblocks = (std::max<int64_t>(n, 1) + 255) / 256;
    const int64_t want = std::max<int64_t>(1, 1024 / cblocks);
    const int64_t by_budget = COL_PART_BUDGET / ((int64_t)COL_SLOTS * std::max<int64_t>(n, 1));
    return (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)COL_CHUNKS_MAX, want, (m + 255) / 256, by_budget}));
}

int64_t col_part_doubles(int64_t m, int64_t n) { return (int64_t)col_pass_chunks(m, n) * COL_SLOTS * n; }

__device__ __forceinline__ double col_point(double lo, double hi, int p)
{
    return lo + (hi - lo) * (double)(p + 1) / (double)(COL_PTS + 1);
}

template <int MODE>
struct ColAcc {
    double s[MODE == 1 ? COL_PTS : 2];
};

template <int MODE>
__device__ __forceinline__ void col_init(ColAcc<MODE> &c)
{
    if constexpr (MODE == 0) {
        c.s[0] = __builtin_huge_val();
        c.s[1] = -__builtin_huge_val();
    } else {
#pragma unroll
        for (int p = 0; p < (MODE == 1 ? COL_PTS : 2); ++p) c.s[p] = 0.0;
    }
}

template <int MODE>
__device__ __forceinline__ void col_term(const ColArgs &a, int64_t j, float av, ColAcc<MODE> &c)
{
    if constexpr (MODE == 0) {
        c.s[0] = fmin(c.s[0], (double)av);
        c.s[1] = fmax(c.s[1], (double)av);
    } else {
        const int q = a.lt.uniform >= 0 ? a.lt.uniform : a.codes[j];
        const int kind = a.lt.kind[q], lev = a.lt.levels[q];
        const double par = (double)a.lt.param[q];
        if constexpr (MODE == 1) {
            const double lo = a.lo[j], hi = a.hi[j];
#pragma unroll
            for (int p = 0; p < COL_PTS; ++p) c.s[p] += loss_g64(kind, lev, par, col_point(lo, hi, p), (double)av);
        } else {
            c.s[0] += loss_l64(kind, lev, par, a.mid[j], (double)av);
        }
    }
}

template <int MODE>
__device__ __forceinline__ void col_merge(ColAcc<MODE> &c, const ColAcc<MODE> &o)
{
    if constexpr (MODE == 0) {
        c.s[0] = fmin(c.s[0], o.s[0]);
        c.s[1] = fmax(c.s[1], o.s[1]);
    } else {
#pragma unroll
        for (int p = 0; p < (MODE == 1 ? COL_PTS : 2); ++p) c.s[p] += o.s[p];
    }
}

template <int MODE>
constexpr int col_nslots() { return MODE == 1 ? COL_PTS : 2; }

// The rows r0 .. r1 - 1 of column j under loss kind KIND (a constant, so
// the loss's code is selected once per column, not per entry and point).
template <int MODE, int KIND>
__device__ __forceinline__ void col_rows(const ColArgs &a, int64_t j, int64_t r0, int64_t r1, int lev, double par,
                                         ColAcc<MODE> &c)
{
    double x[MODE == 1 ? COL_PTS : 1];
    if constexpr (MODE == 1) {
#pragma unroll
        for (int p = 0; p < COL_PTS; ++p) x[p] = col_point(a.lo[j], a.hi[j], p);
    } else {
        x[0] = a.mid[j];
    }
    if constexpr (KIND == L_LOGISTIC) {
        // The labels are +1 and -1, so at each point the term takes one of two
        // values: the rows are counted by label and each value is taken once
        // per column, n+ t(x, +1) + n- t(x, -1) (any other label takes the
        // formula in the loop).  Nothing is held per point during the loop.
        double cnt_p = 0.0, cnt_m = 0.0;
        for (int64_t i = r0; i < r1; ++i) {
            const float av = a.Ap[i * a.ldp + j];
            if (!(av == av)) continue;
            if (av == 1.0f) {
                cnt_p += 1.0;
            } else if (av == -1.0f) {
                cnt_m += 1.0;
            } else {
#pragma unroll
                for (int p = 0; p < (MODE == 1 ? COL_PTS : 1); ++p)
                    c.s[p] += MODE == 1 ? loss_g64(KIND, lev, par, col_point(a.lo[j], a.hi[j], p), (double)av)
                                        : loss_l64(KIND, lev, par, x[0], (double)av);
            }
        }
#pragma unroll
        for (int p = 0; p < (MODE == 1 ? COL_PTS : 1); ++p) {
            const double xp = MODE == 1 ? x[p] : x[0];
            const double tp = MODE == 1 ? loss_g64(KIND, lev, par, xp, 1.0) : loss_l64(KIND, lev, par, xp, 1.0);
            const double tm = MODE == 1 ? loss_g64(KIND, lev, par, xp, -1.0) : loss_l64(KIND, lev, par, xp, -1.0);
            c.s[p] += cnt_p * tp + cnt_m * tm;
        }
        return;
    }
    for (int64_t i = r0; i < r1; ++i) {
        const float av = a.Ap[i * a.ldp + j];
        if (!(av == av)) continue;
        if constexpr (MODE == 1) {
#pragma unroll
            for (int p = 0; p < COL_PTS; ++p) c.s[p] += loss_g64(KIND, lev, par, x[p], (double)av);
        } else {
            c.s[0] += loss_l64(KIND, lev, par, x[0], (double)av);
        }
    }
}

// thread per column, rows of chunk blockIdx.y (coalesced across the threads)
template <int MODE>
__global__ __launch_bounds__(256) void col_pass_dense_kernel(ColArgs a, int64_t per, double *part)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= a.n) return;
    const int64_t r0 = (int64_t)blockIdx.y * per, r1 = min<int64_t>(a.m, r0 + per);
    ColAcc<MODE> c;
    col_init<MODE>(c);
    if constexpr (MODE == 0) {
        for (int64_t i = r0; i < r1; ++i) {
            const float av = a.Ap[i * a.ldp + j];
            if (av == av) col_term<MODE>(a, j, av, c);
        }
    } else {
        const int q = a.lt.uniform >= 0 ? a.lt.uniform : a.codes[j];
        const int lev = a.lt.levels[q];
        const double par = (double)a.lt.param[q];
        switch (a.lt.kind[q]) {
        case L_QUAD: col_rows<MODE, L_QUAD>(a, j, r0, r1, lev, par, c); break;
        case L_HUBER: col_rows<MODE, L_HUBER>(a, j, r0, r1, lev, par, c); break;
        case L_LOGISTIC: col_rows<MODE, L_LOGISTIC>(a, j, r0, r1, lev, par, c); break;
        case L_HINGE: col_rows<MODE, L_HINGE>(a, j, r0, r1, lev, par, c); break;
        default: col_rows<MODE, L_ORDINAL>(a, j, r0, r1, lev, par, c); break;
        }
    }
#pragma unroll
    for (int p = 0; p < col_nslots<MODE>(); ++p) part[((int64_t)blockIdx.y * COL_SLOTS + p) * a.n + j] = c.s[p];
}

// A workgroup takes 64 columns; wavefront w merges the chunks r = w, w + 4,
// ... in order, and the four results are merged in wavefront order.
template <int MODE>
__global__ __launch_bounds__(256) void col_reduce_kernel(const double *part, int32_t R, int64_t n, double *out)
{
    __shared__ double sAcc[4][COL_SLOTS][64];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // scalar: loops over w stay uniform
    const int64_t j = (int64_t)blockIdx.x * 64 + lane;
    ColAcc<MODE> c;
    col_init<MODE>(c);
    if (j < n) {
#pragma unroll 8
        for (int r = w; r < R; r += 4) {
            ColAcc<MODE> o;
#pragma unroll
            for (int p = 0; p < col_nslots<MODE>(); ++p) o.s[p] = part[((int64_t)r * COL_SLOTS + p) * n + j];
            col_merge<MODE>(c, o);
        }
    }
#pragma unroll
    for (int p = 0; p < col_nslots<MODE>(); ++p) sAcc[w][p][lane] = c.s[p];
    __syncthreads();
    if (w != 0 || j >= n) return;
    for (int q = 1; q < 4; ++q) {
        ColAcc<MODE> o;
#pragma unroll
        for (int p = 0; p < col_nslots<MODE>(); ++p) o.s[p] = sAcc[q][p][lane];
        col_merge<MODE>(c, o);
    }
#pragma unroll
    for (int p = 0; p < col_nslots<MODE>(); ++p) out[(int64_t)p * n + j] = c.s[p];
}

// one wavefront per column of the column-grouped copy
template <int MODE>
__global__ __launch_bounds__(256) void col_pass_coo_kernel(ColArgs a, double *out)
{
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (j >= a.n) return;
    ColAcc<MODE> c;
    col_init<MODE>(c);
    for (int32_t e = a.col_ptr[j] + lane; e < a.col_ptr[j + 1]; e += 64) col_term<MODE>(a, j, a.csc_val[e], c);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        ColAcc<MODE> t;
#pragma unroll
        for (int p = 0; p < col_nslots<MODE>(); ++p) t.s[p] = __shfl_xor(c.s[p], o, 64);
        col_merge<MODE>(c, t);
    }
    if (lane == 0)
#pragma unroll
        for (int p = 0; p < col_nslots<MODE>(); ++p) out[(int64_t)p * a.n + j] = c.s[p];
}

template <int MODE>
static hipError_t col_pass(const ColArgs &a, bool coo, double *part, double *out, hipStream_t st)
{
    if (coo) {
        hipLaunchKernelGGL(col_pass_coo_kernel<MODE>, dim3(nblk(a.n, 4)), dim3(256), 0, st, a, out);
    } else {
        const int R = col_pass_chunks(a.m, a.n);
        const int64_t per = (a.m + R - 1) / R;
        hipLaunchKernelGGL(col_pass_dense_kernel<MODE>, dim3(nblk(a.n), R), dim3(256), 0, st, a, per, part);
        hipLaunchKernelGGL(col_reduce_kernel<MODE>, dim3(nblk(a.n, 64)), dim3(256), 0, st, part, R, a.n, out);
    }
    return hipGetLastError();
}

hipError_t launch_col_pass(const ColArgs &a, int mode, bool coo, double *part, double *out, hipStream_t st)
{
    switch (mode) {
    case 0: return col_pass<0>(a, coo, part, out, st);
    case 1: return col_pass<1>(a, coo, part, out, st);
    default: return col_pass<2>(a, coo, part, out, st);
    }
}

// init: lo = min - 1, hi = max + 1 (out: mode 0).  Step (out: mode 1): the
// bracket becomes the sub-interval ending at the first of its points where
// the derivative sum is not negative (the rule of a bisection step, at
// COL_PTS points at once): the minimum lies at or below that point and above
// the one before it.
__global__ void bracket_kernel(double *lo, double *hi, double *mid, const double *out, const int32_t *count, int64_t n,
                               bool init)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    if (init) {
        if (count[j] > 0) {
            lo[j] = out[j] - 1.0;
            hi[j] = out[n + j] + 1.0;
        } else {
            lo[j] = hi[j] = 0.0;
        }
    } else {
        const double l = lo[j], h = hi[j];
        double nl = col_point(l, h, COL_PTS - 1), nh = h;
        for (int p = COL_PTS - 1; p >= 0; --p) {
            if (!(out[(int64_t)p * n + j] < 0.0)) {
                nh = col_point(l, h, p);
                nl = p > 0 ? col_point(l, h, p - 1) : l;
            }
        }
        lo[j] = nl;
        hi[j] = nh;
    }
    mid[j] = 0.5 * (lo[j] + hi[j]);
}

hipError_t launch_bracket(double *lo, double *hi, double *mid, const double *out, const int32_t *count, int64_t n,
                          bool init, hipStream_t st)
{
    hipLaunchKernelGGL(bracket_kernel, dim3(nblk(n)), dim3(256), 0, st, lo, hi, mid, out, count, n, init);
    return hipGetLastError();
}

__global__ void scaling_finish_kernel(const double *mid, const double *out, const int32_t *count, int64_t n, float *mu,
                                      float *sigma2)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const int c = count[j];
    mu[j] = c > 0 ? (float)mid[j] : 0.0f;
    const double S = out[j];
    sigma2[j] = (c >= 2 && S > 0.0) ? (float)(S / (double)(c - 1)) : 1.0f;
}

hipError_t launch_scaling_finish(const double *mid, const double *out, const int32_t *count, int64_t n, float *mu,
                                 float *sigma2, hipStream_t st)
{
    hipLaunchKernelGGL(scaling_finish_kernel, dim3(nblk(n)), dim3(256), 0, st, mid, out, count, n, mu, sigma2);
    return hipGetLastError();
}

__global__ void svd_scales_kernel(const float *mu, const float *sigma2, const int32_t *count, int64_t m, int64_t n,
                                  float *cs, float *mu0)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const int c = count[j];
    const double sig = sigma2 ? sqrt((double)sigma2[j]) : 1.0;
    cs[j] = (c > 0 && sig > 0.0) ? (float)((double)m / (sig * (double)c)) : 0.0f;
    mu0[j] = mu ? mu[j] : 0.0f;
}

hipError_t launch_svd_scales(const float *mu, const float *sigma2, const int32_t *count, int64_t m, int64_t n,
                             float *cs, float *mu0, hipStream_t st)
{
    hipLaunchKernelGGL(svd_scales_kernel, dim3(nblk(n)), dim3(256), 0, st, mu, sigma2, count, m, n, cs, mu0);
    return hipGetLastError();
}

__global__ void to_float_scaled_kernel(const double *src, int64_t rows, int32_t b, int32_t cols,
                                       const float *rowscale, float *dst, int64_t ldd, int32_t col0)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= rows * cols) return;
    const int64_t i = t / cols;
    const int c = (int)(t % cols);
    const double sc = rowscale ? sqrt((double)rowscale[i]) : 1.0;
    dst[i * ldd + col0 + c] = (float)(src[i * b + c] * sc);
}

hipError_t launch_to_float_scaled(const double *src, int64_t rows, int32_t b, int32_t cols, const float *rowscale,
                                  float *dst, int64_t ldd, int32_t col0, hipStream_t st)
{
    if (rows * cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_float_scaled_kernel, dim3(nblk(rows * cols)), dim3(256), 0, st, src, rows, b, cols, rowscale,
                       dst, ldd, col0);
    return hipGetLastError();
}

__global__ void fill_column_kernel(float *dst, int64_t rows, int64_t ldd, int32_t col, float value,
                                   const float *value_vec)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < rows) dst[i * ldd + col] = value_vec ? value_vec[i] : value;
}

hipError_t launch_fill_column(float *dst, int64_t rows, int64_t ldd, int32_t col, float value,
                              const float *value_vec, hipStream_t st)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_column_kernel, dim3(nblk(rows)), dim3(256), 0, st, dst, rows, ldd, col, value, value_vec);
    return hipGetLastError();
}

__global__ void to_double_kernel(const float *src, int64_t len, double *dst)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < len) dst[t] = (double)src[t];
}

hipError_t launch_to_double(const float *src, int64_t len, double *dst, hipStream_t st)
{
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_double_kernel, dim3(nblk(len)), dim3(256), 0, st, src, len, dst);
    return hipGetLastError();
}

}  // namespace glrm
