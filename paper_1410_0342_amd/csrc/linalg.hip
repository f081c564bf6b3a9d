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
    for (int l = 0; l < a.k; ++l) z += (double)a.X[i * a.k + l] * (double)a.Y[j * a.k + l];
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

constexpr int LA_Q = LA_MAXB / 16;   // outputs per thread along the block

// out (m x b) = alpha V B.  A workgroup owns 16 rows; 64-column slices of V and
// of B go through LDS; thread (r, cl) accumulates row r's outputs cl + 16 q.
__global__ __launch_bounds__(256) void dense_apply_kernel(const float *V, int64_t m, int64_t n, int64_t ldp,
                                                          const double *B, int32_t b, double alpha, double *out)
{
    __shared__ float sV[16][65];
    __shared__ double sB[64][LA_MAXB + 1];
    const int t = threadIdx.x, r = t >> 4, cl = t & 15;
    const int64_t i0 = (int64_t)blockIdx.x * 16;
    double acc[LA_Q];
#pragma unroll
    for (int q = 0; q < LA_Q; ++q) acc[q] = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += 64) {
        for (int e = t; e < 16 * 64; e += 256) {
            const int rr = e >> 6, jj = e & 63;
            const int64_t i = i0 + rr, j = j0 + jj;
            sV[rr][jj] = (i < m && j < n) ? V[i * ldp + j] : 0.0f;
        }
        for (int e = t; e < 64 * b; e += 256) {
            const int jj = e / b, c = e % b;
            const int64_t j = j0 + jj;
            sB[jj][c] = j < n ? B[j * b + c] : 0.0;
        }
        __syncthreads();
        const int jn = (int)min<int64_t>(64, n - j0);
        for (int jj = 0; jj < jn; ++jj) {
            const double v = (double)sV[r][jj];
#pragma unroll
            for (int q = 0; q < LA_Q; ++q) {
                const int c = cl + 16 * q;
                if (c < b) acc[q] += v * sB[jj][c];
            }
        }
        __syncthreads();
    }
    const int64_t i = i0 + r;
    if (i < m) {
#pragma unroll
        for (int q = 0; q < LA_Q; ++q) {
            const int c = cl + 16 * q;
            if (c < b) out[i * b + c] = alpha * acc[q];
        }
    }
}

// One vector (b = 1): out_i = alpha sum_j V_ij x_j, one wavefront per row
// (lane l takes the columns l, l + 64, ..., coalesced), the lanes' sums
// combined by a butterfly.
__global__ __launch_bounds__(256) void dense_gemv_kernel(const float *V, int64_t m, int64_t n, int64_t ldp,
                                                         const double *x, double alpha, double *out)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < m; i += nw) {
        const float *row = V + i * ldp;
        double acc = 0.0;
        for (int64_t j = lane; j < n; j += 64) acc += (double)row[j] * x[j];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) out[i] = alpha * acc;
    }
}

hipError_t launch_dense_apply(const float *V, int64_t m, int64_t n, int64_t ldp, const double *B, int32_t b,
                              double alpha, double *out, hipStream_t st)
{
    if (b < 1 || b > LA_MAXB) return hipErrorInvalidValue;
    if (b == 1) {
        const int64_t blocks = std::min<int64_t>((m + 3) / 4, 8192);
        hipLaunchKernelGGL(dense_gemv_kernel, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, st, V, m, n,
                           ldp, B, alpha, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(dense_apply_kernel, dim3(nblk(m, 16)), dim3(256), 0, st, V, m, n, ldp, B, b, alpha, out);
    return hipGetLastError();
}

// Partials of V^T Q: workgroup (column block of 16, row chunk); rows go through
// LDS in slices of 64.
__global__ __launch_bounds__(256) void dense_apply_t_kernel(const float *V, int64_t m, int64_t n, int64_t ldp,
                                                            const double *Q, int32_t b, int64_t per, double *part)
{
    __shared__ float sV[64][17];
    __shared__ double sQ[64][LA_MAXB + 1];
    const int t = threadIdx.x, jj = t >> 4, cl = t & 15;
    const int64_t j0 = (int64_t)blockIdx.x * 16;
    const int64_t r0 = (int64_t)blockIdx.y * per, r1 = min<int64_t>(m, r0 + per);
    double acc[LA_Q];
#pragma unroll
    for (int q = 0; q < LA_Q; ++q) acc[q] = 0.0;
    for (int64_t i0 = r0; i0 < r1; i0 += 64) {
        for (int e = t; e < 64 * 16; e += 256) {
            const int ii = e >> 4, c = e & 15;
            const int64_t i = i0 + ii, j = j0 + c;
            sV[ii][c] = (i < r1 && j < n) ? V[i * ldp + j] : 0.0f;
        }
        for (int e = t; e < 64 * b; e += 256) {
            const int ii = e / b, c = e % b;
            const int64_t i = i0 + ii;
            sQ[ii][c] = i < r1 ? Q[i * b + c] : 0.0;
        }
        __syncthreads();
        const int in_ = (int)min<int64_t>(64, r1 - i0);
        for (int ii = 0; ii < in_; ++ii) {
            const double v = (double)sV[ii][jj];
#pragma unroll
            for (int q = 0; q < LA_Q; ++q) {
                const int c = cl + 16 * q;
                if (c < b) acc[q] += v * sQ[ii][c];
            }
        }
        __syncthreads();
    }
    const int64_t j = j0 + jj;
    if (j < n) {
#pragma unroll
        for (int q = 0; q < LA_Q; ++q) {
            const int c = cl + 16 * q;
            if (c < b) part[((int64_t)blockIdx.y * n + j) * b + c] = acc[q];
        }
    }
}

// out[e] = alpha * sum_p part[p][e] over p = 0..np-1, in that order.
__global__ void reduce_parts_kernel(const double *part, int32_t np, int64_t len, double alpha, double *out)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= len) return;
    double s = 0.0;
    for (int p = 0; p < np; ++p) s += part[(int64_t)p * len + e];
    out[e] = alpha * s;
}

int dense_apply_t_chunks(int64_t m, int64_t n)
{
    const int64_t cblocks = (n + 15) / 16;
    const int64_t want = std::max<int64_t>(1, 2048 / cblocks);
    return (int)std::min<int64_t>({want, (int64_t)LA_TCHUNKS, std::max<int64_t>(1, (m + 63) / 64)});
}

// One vector (b = 1): partials of V^T q per row chunk.  A workgroup takes 64
// columns (lane -> column, coalesced) and a chunk of rows, its four
// wavefronts every fourth row; the four sums are combined in order.
__global__ __launch_bounds__(256) void dense_gemv_t_kernel(const float *V, int64_t m, int64_t n, int64_t ldp,
                                                           const double *q, int64_t per, double *part)
{
    __shared__ double sAcc[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + lane;
    const int64_t r0 = (int64_t)blockIdx.y * per, r1 = min<int64_t>(m, r0 + per);
    double acc = 0.0;
    if (j < n)
        for (int64_t i = r0 + w; i < r1; i += 4) acc += (double)V[i * ldp + j] * q[i];
    sAcc[w][lane] = acc;
    __syncthreads();
    if (w == 0 && j < n) part[(int64_t)blockIdx.y * n + j] = ((sAcc[0][lane] + sAcc[1][lane]) + sAcc[2][lane]) + sAcc[3][lane];
}

hipError_t launch_dense_apply_t(const float *V, int64_t m, int64_t n, int64_t ldp, const double *Q, int32_t b,
                                double alpha, double *part, double *out, hipStream_t st)
{
    if (b < 1 || b > LA_MAXB) return hipErrorInvalidValue;
    if (b == 1) {
        // row chunks: enough workgroups to fill the device, partials within LA_TCHUNKS n
        const int64_t cblocks = (n + 63) / 64;
        const int ch = (int)std::min<int64_t>({(int64_t)LA_TCHUNKS, std::max<int64_t>(1, 4096 / cblocks),
                                               std::max<int64_t>(1, (m + 255) / 256)});
        const int64_t per = (m + ch - 1) / ch;
        hipLaunchKernelGGL(dense_gemv_t_kernel, dim3((unsigned)cblocks, ch), dim3(256), 0, st, V, m, n, ldp, Q, per,
                           part);
        hipLaunchKernelGGL(reduce_parts_kernel, dim3(nblk(n)), dim3(256), 0, st, part, ch, n, alpha, out);
        return hipGetLastError();
    }
    const int ch = dense_apply_t_chunks(m, n);
    const int64_t per = (m + ch - 1) / ch;
    hipLaunchKernelGGL(dense_apply_t_kernel, dim3(nblk(n, 16), ch), dim3(256), 0, st, V, m, n, ldp, Q, b, per,
                       part);
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(nblk(n * b)), dim3(256), 0, st, part, ch, n * b, alpha, out);
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
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
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

constexpr int TALL_ROWS = 1024;     // rows per workgroup of U^T B

int tall_tmul_blocks(int64_t rows) { return (int)std::min<int64_t>(4096, std::max<int64_t>(1, (rows + TALL_ROWS - 1) / TALL_ROWS)); }

// part[blk][l b + c] = sum over the workgroup's rows of U[i, l] B[i, c]
template <typename TU, typename TB>
__global__ __launch_bounds__(256) void tall_tmul_kernel(const TU *U, int64_t rows, int32_t k, int64_t ldu,
                                                        const TB *B, int64_t ldb, int32_t b, int64_t per,
                                                        double *part)
{
    const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min<int64_t>(rows, i0 + per);
    const int np = k * b;
    for (int p0 = 0; p0 < np; p0 += 256) {
        const int p = p0 + threadIdx.x;
        if (p < np) {
            const int l = p / b, c = p % b;
            double acc = 0.0;
            for (int64_t i = i0; i < i1; ++i) acc += (double)U[i * ldu + l] * (double)B[i * ldb + c];
            part[(int64_t)blockIdx.x * np + p] = acc;
        }
    }
}

template <typename TU, typename TB>
static hipError_t tall_tmul(const TU *U, int64_t rows, int32_t k, int64_t ldu, const TB *B, int64_t ldb, int32_t b,
                            double *part, double *out, hipStream_t st)
{
    const int nb = tall_tmul_blocks(rows);
    const int64_t per = (rows + nb - 1) / nb;
    hipLaunchKernelGGL((tall_tmul_kernel<TU, TB>), dim3(nb), dim3(256), 0, st, U, rows, k, ldu, B, ldb, b, per, part);
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(nblk((int64_t)k * b)), dim3(256), 0, st, part, nb, (int64_t)k * b,
                       1.0, out);
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
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(1), dim3(256), 0, st, part, SUMSQ_BLOCKS, (int64_t)1, 1.0, nrm2);
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

int col_pass_chunks(int64_t m, int64_t n)
{
    const int64_t by_budget = COL_PART_BUDGET / ((int64_t)COL_SLOTS * std::max<int64_t>(n, 1));
    return (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)COL_CHUNKS_MAX, (m + 255) / 256, by_budget}));
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

template <int MODE>
__global__ void col_reduce_kernel(const double *part, int32_t R, int64_t n, double *out)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    ColAcc<MODE> c;
    col_init<MODE>(c);
    for (int r = 0; r < R; ++r) {
        ColAcc<MODE> o;
#pragma unroll
        for (int p = 0; p < col_nslots<MODE>(); ++p) o.s[p] = part[((int64_t)r * COL_SLOTS + p) * n + j];
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
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
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
        hipLaunchKernelGGL(col_reduce_kernel<MODE>, dim3(nblk(a.n)), dim3(256), 0, st, part, R, a.n, out);
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
