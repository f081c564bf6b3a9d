// Imputation (Section 5.3): every entry of the table decoded from the fitted
// factors, a_hat_ij = argmin over the column's data domain of L_j(x_i . y_j, a).
//
// The pass is bound by its m x n store.  Each lane owns one column j and keeps
// y_j in registers; a workgroup walks a chunk of rows, and every row's x_i is
// the same for the whole wavefront, so it comes in through scalar loads and
// feeds the lanes' multiply-adds as a scalar operand.
//
// Stores: HBM takes whole 128-byte lines far faster than parts of lines, and a
// row of 4n bytes starts on a line boundary only when 4n is a multiple of 128.
// A contiguous table of at most 1024 columns whose rows are not line-aligned
// runs one workgroup per row width (4 wavefronts up to 256 columns, 16 up to
// 1024), so the workgroup stages SB rows in LDS and stores their flat range
// with line-aligned wavefront stores; other tables store each row's 64 columns
// per wavefront directly, in workgroups of 256 columns.  The every-entry form
// stores non-temporally (the table is not read back here); the missing-only
// form measured faster with plain stores.
#include <algorithm>
#include <utility>

#include "glrm_device.h"
#include "impute.h"

namespace glrm {

// The decoded value for the three domains: real (quadratic, Huber: the product
// itself), Boolean (logistic, hinge: +1 above zero, -1 otherwise, so a tie at
// zero takes the smaller value) and ordinal (the nearest level, clamped to
// 1..levels, a half-way tie taking the lower one: stepping from level a to a+1
// lowers the ordinal hinge only while a < u - 1/2).  u - 0.5f is exact wherever
// the clamp does not decide the result.
__device__ __forceinline__ float decode_entry(float u, int kind, float levels)
{
    const float boolean = u > 0.0f ? 1.0f : -1.0f;
    const float ordinal = fminf(fmaxf(ceilf(u - 0.5f), 1.0f), levels);
    return kind <= L_HUBER ? u : (kind <= L_HINGE ? boolean : ordinal);
}

// Rows of the table loaded ahead in the missing-only form (clamped to the
// chunk, so the loads past its end repeat its last row and stay in bounds).
template <int RB>
__device__ __forceinline__ void load_rows(const float *__restrict__ A, const uint8_t *__restrict__ mask, int64_t lda,
                                          int64_t ib, int64_t i1, int64_t jc, float (&av)[RB], uint8_t (&obs)[RB])
{
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int64_t o = (ib + r < i1 ? ib + r : i1 - 1) * lda + jc;
        obs[r] = mask[o];
        av[r] = A[o];
    }
}

constexpr int SB = 16;   // rows staged per flat store

// The staged rows of the flat form (SB rows of at most W columns).
template <int W>
__device__ __forceinline__ float *stage_tile()
{
    __shared__ float tile[SB * W];
    return tile;
}

template <bool NT>
__device__ __forceinline__ void store_entry(float *p, float v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// KEEP: observed entries (mask != 0) keep A_ij (the missing-only form).
// FW: 0 for direct stores (workgroups of 256 columns); otherwise the table is
// contiguous (ldh == n) with n <= 64 FW, a workgroup of FW wavefronts spans a
// row, and rows go through LDS and out as one flat, line-aligned range per SB
// rows.
template <int K, bool KEEP, int FW>
__global__ __launch_bounds__(FW == 0 ? 256 : 64 * FW) void impute_kernel(ImputeArgs a, const float *__restrict__ X,
                                                     const float *__restrict__ Y, const float *__restrict__ A,
                                                     const uint8_t *__restrict__ mask, float *__restrict__ out)
{
    constexpr bool NT = !KEEP;
    constexpr bool FLAT = FW != 0;
    constexpr int TB = FLAT ? 64 * FW : 256;   // threads per workgroup
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t ncb = FLAT ? 1 : (a.n + 255) >> 8;
    const int64_t cb = blockIdx.x % ncb, chunk = blockIdx.x / ncb;
    const int64_t j = cb * 256 + w * 64 + lane;
    const bool live = j < a.n;
    const int64_t jc = live ? j : a.n - 1;

    float y[K];
#pragma unroll
    for (int l = 0; l < K; ++l) y[l] = Y[jc * K + l];
    // this column's loss, picked from the table by its code
    const int code = a.codes[jc];
    int kind = a.lt.kind[0];
    float levels = (float)a.lt.levels[0];
#pragma unroll
    for (int q = 1; q < MAX_LOSSES; ++q)
        if (code == q) {
            kind = a.lt.kind[q];
            levels = (float)a.lt.levels[q];
        }
    // Stores and loads share one completion counter, so a wait for y_j inside
    // the row loop would also wait for every store issued before it: wait once
    // here.  The missing-only form loads the table one batch of rows ahead, so
    // its wait for a batch leaves the stores issued since in flight; the
    // barriers around the staged rows wait on LDS only, for the same reason.
    __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
#pragma unroll
    for (int l = 0; l < K; ++l) asm volatile("" : "+v"(y[l]));   // y_j is in registers from here on
    constexpr int RB = 4;
    const int64_t i0 = chunk * a.rows_per_block;
    const int64_t i1 = i0 + a.rows_per_block < a.m ? i0 + a.rows_per_block : a.m;
    float av[RB], avn[RB];
    uint8_t obs[RB], obsn[RB];
    if constexpr (KEEP) load_rows<RB>(A, mask, a.lda, i0, i1, jc, av, obs);
    for (int64_t sb = i0; sb < i1; sb += SB) {
        const int64_t se = sb + SB < i1 ? sb + SB : i1;
        for (int64_t ib = sb; ib < se; ib += RB) {
            if constexpr (KEEP) load_rows<RB>(A, mask, a.lda, ib + RB, i1, jc, avn, obsn);
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int64_t i = ib + r;
                if (i >= se) break;
                const float *xr = X + i * K;
                float u = 0.0f;
#pragma unroll
                for (int l = 0; l < K; ++l) u = __builtin_fmaf(xr[l], y[l], u);
                float v = decode_entry(u, kind, levels);
                if constexpr (KEEP) v = obs[r] != 0 ? av[r] : v;
                if constexpr (FLAT) {
                    if (live) stage_tile<TB>()[(i - sb) * a.n + j] = v;
                } else {
                    if (live) store_entry<NT>(&out[i * a.ldh + j], v);
                }
            }
            if constexpr (KEEP) {
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    av[r] = avn[r];
                    obs[r] = obsn[r];
                }
            }
        }
        if constexpr (FLAT) {
            // the staged rows are out[sb * n, se * n): store it from the line
            // that holds its first entry, TB consecutive entries per pass
            lds_barrier();
            const int64_t f0 = sb * a.n, f1 = se * a.n;
            for (int64_t t = (f0 & ~(int64_t)31) + threadIdx.x; t < f1; t += TB)
                if (t >= f0) store_entry<NT>(&out[t], stage_tile<TB>()[t - f0]);
            lds_barrier();
        }
    }
}

// Observed entries of a row-sorted COO list written over the decoded table.
// Indices outside the table are skipped (the host validates them beforehand).
__global__ __launch_bounds__(256) void scatter_observed_kernel(int64_t nnz, int64_t m, int64_t n, int64_t ldh,
                                                               const int32_t *__restrict__ row,
                                                               const int32_t *__restrict__ col,
                                                               const float *__restrict__ val, float *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nnz) return;
    const int64_t r = row[e], c = col[e];
    if (r >= 0 && r < m && c >= 0 && c < n) out[r * ldh + c] = val[e];
}

// The launch form: staged only where rows do not start on line boundaries
// (aligned rows measured faster stored directly), and only while one
// workgroup spans a row.
static int flat_waves(const ImputeArgs &a)
{
    if (a.ldh != a.n || (a.n % 32) == 0 || a.n > 1024) return 0;
    return a.n <= 256 ? 4 : 16;
}

int impute_rows_per_block(int64_t m, int64_t n)
{
    // about eight 256-thread workgroups per CU over the whole table (as many
    // threads with the wider ones), at least 16 rows each
    const int64_t ncb = (n + 255) / 256;
    const int64_t chunks = std::max<int64_t>(1, (IMPUTE_TARGET_BLOCKS + ncb - 1) / ncb);
    return (int)std::max<int64_t>(16, (m + chunks - 1) / chunks);
}

template <int K, bool KEEP, int FW>
static void launch_form(const ImputeArgs &a, const float *X, const float *Y, const float *A, const uint8_t *mask,
                        float *out, hipStream_t st)
{
    // a staged workgroup spans all of a row's 256-column blocks, so a chunk of
    // rows is one workgroup of as many threads
    const int64_t ncb = FW == 0 ? (a.n + 255) / 256 : 1;
    const int64_t chunks = (a.m + a.rows_per_block - 1) / a.rows_per_block;
    hipLaunchKernelGGL((impute_kernel<K, KEEP, FW>), dim3((unsigned)(ncb * chunks)), dim3(FW == 0 ? 256 : 64 * FW), 0,
                       st, a, X, Y, A, mask, out);
}

// One instance per rank, so a row of X is a fixed run of scalar loads.
template <int K>
static hipError_t launch_k(const ImputeArgs &a, const float *X, const float *Y, const float *A, const uint8_t *mask,
                           float *out, hipStream_t st)
{
    const int fw = flat_waves(a);
    if (a.keep_observed) {
        if (fw == 4) launch_form<K, true, 4>(a, X, Y, A, mask, out, st);
        else if (fw == 16) launch_form<K, true, 16>(a, X, Y, A, mask, out, st);
        else launch_form<K, true, 0>(a, X, Y, A, mask, out, st);
    } else {
        if (fw == 4) launch_form<K, false, 4>(a, X, Y, A, mask, out, st);
        else if (fw == 16) launch_form<K, false, 16>(a, X, Y, A, mask, out, st);
        else launch_form<K, false, 0>(a, X, Y, A, mask, out, st);
    }
    return hipGetLastError();
}

template <int... Ks>
static hipError_t launch_rank(const ImputeArgs &a, const float *X, const float *Y, const float *A,
                              const uint8_t *mask, float *out, hipStream_t st, std::integer_sequence<int, Ks...>)
{
    hipError_t e = hipErrorInvalidValue;
    ((a.k == Ks + 1 ? (e = launch_k<Ks + 1>(a, X, Y, A, mask, out, st), 0) : 0), ...);
    return e;
}

hipError_t launch_impute(const ImputeArgs &a, const float *X, const float *Y, const float *A, const uint8_t *mask,
                         float *out, hipStream_t st)
{
    return launch_rank(a, X, Y, A, mask, out, st, std::make_integer_sequence<int, IMPUTE_MAX_K>{});
}

// ---- tables with multi-dimensional losses (Section 6) ------------------------
// One thread per entry (i, j) of the table: u_l = x_i . (row fcol[j] + l of
// Y), each a float32 fused multiply-add chain over the rank, and the value
// that minimizes the feature's loss (Section 5.3):
//   categorical   the label of the largest u_l (the first of equal ones): the
//                 one-vs-all loss is the largest part of the sum minus a
//                 strictly decreasing function of u_a, so its argmin is the argmax
//   ordinal       the level a minimizing sum_{l < a-1} (1 - u_l)_+ +
//                 sum_{l >= a-1} (1 + u_l)_+; from a to a + 1 the sum changes by
//                 (1 - u_{a-1})_+ - (1 + u_{a-1})_+, so a running sum of those
//                 steps ranks the levels (the first of equal minima)
//   other kinds   the scalar rules of decode_entry
__global__ __launch_bounds__(256) void impute_md_kernel(ImputeMDArgs a, const float *__restrict__ X,
                                                        const float *__restrict__ Y, const float *__restrict__ A,
                                                        const uint8_t *__restrict__ mask, float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= a.m * a.nf) return;
    const int64_t i = t / a.nf, j = t - i * a.nf;
    if (a.keep_observed && mask[i * a.lda + j] != 0) {
        out[i * a.ldh + j] = A[i * a.lda + j];
        return;
    }
    const float *x = X + i * a.k;
    const int kind = a.fkind[j], lev = a.flev[j];
    const float *y0 = Y + (int64_t)a.fcol[j] * a.k;
    auto dot = [&](int l) {
        const float *y = y0 + (int64_t)l * a.k;
        float u = 0.0f;
        for (int c = 0; c < a.k; ++c) u = __builtin_fmaf(x[c], y[c], u);
        return u;
    };
    float v;
    if (kind == L_CATEGORICAL) {
        int best = 0;
        float bu = dot(0);
        for (int l = 1; l < lev; ++l) {
            const float u = dot(l);
            if (u > bu) { bu = u; best = l; }
        }
        v = (float)(best + 1);
    } else if (kind == L_MORDINAL) {
        int best = 1;
        float D = 0.0f, bD = 0.0f;
        for (int l = 0; l < lev - 1; ++l) {
            const float u = dot(l);
            D += fmaxf(1.0f - u, 0.0f) - fmaxf(1.0f + u, 0.0f);
            if (D < bD) { bD = D; best = l + 2; }
        }
        v = (float)best;
    } else {
        v = decode_entry(dot(0), kind, (float)lev);
    }
    out[i * a.ldh + j] = v;
}

hipError_t launch_impute_md(const ImputeMDArgs &a, const float *X, const float *Y, const float *A, const uint8_t *mask,
                            float *out, hipStream_t st)
{
    const int64_t total = a.m * a.nf;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(impute_md_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a, X, Y, A, mask,
                       out);
    return hipGetLastError();
}

hipError_t launch_scatter_observed(int64_t nnz, int64_t m, int64_t n, int64_t ldh, const int32_t *row,
                                   const int32_t *col, const float *val, float *out, hipStream_t st)
{
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_observed_kernel, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st, nnz, m, n,
                       ldh, row, col, val, out);
    return hipGetLastError();
}

}  // namespace glrm
