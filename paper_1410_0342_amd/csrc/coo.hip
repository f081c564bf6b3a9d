// Sparse path: the observed set handed over as a row-sorted COO list.
//
// Set-up builds, in the workspace, the row pointers of the row-compressed view
// (the input itself, since it is row-sorted) and a column-grouped copy (row
// index and value of every entry, ordered by column then row) with a stable
// radix sort, so every later reduction has a fixed order.
//
// The X half-step walks rows, the Y half-step walks columns: Section 7.2
// defines the Y update as the X update on the transposed problem, and a walk
// that owns its row (column) can take the step, re-evaluate the trial point
// and decide without any cross-workgroup exchange.  A wavefront owns one row
// (column) at a time; inside it, groups of kp/4 lanes share one entry, each
// lane holding four coordinates, so a factor row is one coalesced
// 16-byte-per-lane gather and z = x_i . y_j is a short butterfly over the group.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "coo.h"
#include "glrm_kernels.h"

namespace glrm {

constexpr int CW = 4;              // wavefronts per workgroup
constexpr int COO_MAX_WAVES = 8192;

static int64_t rup(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// ---- layout ------------------------------------------------------------------
void coo_layout(const glrm_data *d, int kp, CooLayout &cl)
{
    cl = CooLayout();
    cl.m = d->m; cl.n = d->n; cl.nnz = d->nnz; cl.kp = kp;
    const int64_t nnz = std::max<int64_t>(d->nnz, 1);
    auto take = [&](size_t bytes) { size_t o = cl.total; cl.total += (size_t)rup((int64_t)bytes, 256); return o; };
    cl.row_ptr = take(sizeof(int32_t) * (d->m + 1));
    cl.col_ptr = take(sizeof(int32_t) * (d->n + 1));
    cl.csc_row = take(sizeof(int32_t) * nnz);
    cl.csc_val = take(sizeof(float) * nnz);
    cl.perm_in = take(sizeof(int32_t) * nnz);
    cl.perm_out = take(sizeof(int32_t) * nnz);
    cl.keys_out = take(sizeof(int32_t) * nnz);
    size_t tb = 0;
    int bits = 1;
    while ((int64_t(1) << bits) < d->n) ++bits;
    hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (const int *)nullptr, (int *)nullptr, (const int *)nullptr,
                                       (int *)nullptr, (int)nnz, 0, bits, (hipStream_t)0);
    cl.sort_tmp_bytes = tb;
    cl.sort_tmp = take(tb);
    cl.flags = take(sizeof(int32_t) * 4);
    cl.part_bytes = (sizeof(double) * 2 + sizeof(int32_t) * 2) * COO_MAX_WAVES;
    cl.part = take(cl.part_bytes);
    cl.xs = take(sizeof(float) * d->m * kp);
    cl.ys = take(sizeof(float) * d->n * kp);
}

struct CooPtrs {
    int32_t *row_ptr, *col_ptr, *csc_row, *perm_in, *perm_out, *keys_out, *flags;
    float *csc_val, *xs, *ys;
    double *partA, *partB;
    int32_t *ipartA, *ipartB;
    void *sort_tmp;
};

static CooPtrs ptrs(const CooLayout &cl, char *b)
{
    CooPtrs p;
    p.row_ptr = (int32_t *)(b + cl.row_ptr);
    p.col_ptr = (int32_t *)(b + cl.col_ptr);
    p.csc_row = (int32_t *)(b + cl.csc_row);
    p.csc_val = (float *)(b + cl.csc_val);
    p.perm_in = (int32_t *)(b + cl.perm_in);
    p.perm_out = (int32_t *)(b + cl.perm_out);
    p.keys_out = (int32_t *)(b + cl.keys_out);
    p.sort_tmp = b + cl.sort_tmp;
    p.flags = (int32_t *)(b + cl.flags);
    char *q = b + cl.part;
    p.partA = (double *)q;
    p.partB = p.partA + COO_MAX_WAVES;
    p.ipartA = (int32_t *)(p.partB + COO_MAX_WAVES);
    p.ipartB = p.ipartA + COO_MAX_WAVES;
    p.xs = (float *)(b + cl.xs);
    p.ys = (float *)(b + cl.ys);
    return p;
}

CooView coo_view(const CooLayout &cl, char *base)
{
    CooPtrs p = ptrs(cl, base);
    return CooView{p.row_ptr, p.col_ptr, p.csc_row, p.csc_val};
}

// perm_out[p] is the row-order position of the p-th entry of the column-grouped copy
const int32_t *coo_perm(const CooLayout &cl, char *base) { return ptrs(cl, base).perm_out; }

// ---- set-up kernels ------------------------------------------------------------

// Order and range check of the COO list; flags[0] != 0 on any violation.
__global__ void coo_validate_kernel(const int32_t *row, const int32_t *col, int64_t nnz, int64_t m, int64_t n,
                                    int32_t *flags)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nnz) return;
    const int32_t r = row[e], c = col[e];
    bool bad = r < 0 || r >= m || c < 0 || c >= n;
    if (e > 0) {
        const int32_t r0 = row[e - 1], c0 = col[e - 1];
        bad = bad || r0 > r || (r0 == r && c0 >= c);
    }
    if (bad) atomicOr(&flags[0], 1);
}

// Segment pointers of a sorted key list: ptr[i] = first position whose key is
// >= i, for i = 0..len, by binary search.  The cost is bounded for any input;
// an unsorted list gives meaningless pointers that are never used, because the
// validation kernel reports it and set-up fails.
__global__ void seg_ptr_kernel(const int32_t *keys, int64_t nnz, int64_t len, int32_t *ptr)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i > len) return;
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)keys[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    ptr[i] = (int32_t)lo;
}

__global__ void seg_count_kernel(const int32_t *ptr, int64_t len, int32_t *count)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) count[i] = ptr[i + 1] - ptr[i];
}

__global__ void iota_kernel(int32_t *p, int64_t len)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) p[i] = (int32_t)i;
}

__global__ void gather_csc_kernel(const int32_t *perm, const int32_t *row, const float *val, int64_t nnz,
                                  int32_t *csc_row, float *csc_val)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < nnz) {
        const int32_t e = perm[p];
        csc_row[p] = row[e];
        csc_val[p] = val[e];
    }
}

// Padded copy of a factor: dst (rows x kp) from src (rows x k).
__global__ void pad_factor_kernel(const float *src, int64_t rows, int32_t k, int32_t kp, float *dst)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= rows * kp) return;
    const int64_t i = t / kp;
    const int c = (int)(t % kp);
    dst[t] = c < k ? src[i * k + c] : 0.0f;
}

static unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

int coo_prepare(const glrm_data *d, int kp, const CooLayout &cl, char *base, int32_t *row_count,
                int32_t *col_count, hipStream_t st)
{
    (void)kp;
    CooPtrs p = ptrs(cl, base);
    const int64_t nnz = d->nnz, m = d->m, n = d->n;
    hipError_t e;
    if ((e = launch_fill_i32(p.flags, 4, 0, st)) != hipSuccess)
        return set_error(GLRM_EHIP, "clearing the validation flags: %s", hipGetErrorString(e));
    if (nnz > 0) hipLaunchKernelGGL(coo_validate_kernel, dim3(nblk(nnz)), dim3(256), 0, st, d->row, d->col, nnz, m, n, p.flags);
    hipLaunchKernelGGL(seg_ptr_kernel, dim3(nblk(m + 1)), dim3(256), 0, st, d->row, nnz, m, p.row_ptr);
    hipLaunchKernelGGL(seg_count_kernel, dim3(nblk(m)), dim3(256), 0, st, p.row_ptr, m, row_count);
    if (nnz > 0) {
        hipLaunchKernelGGL(iota_kernel, dim3(nblk(nnz)), dim3(256), 0, st, p.perm_in, nnz);
        int bits = 1;
        while ((int64_t(1) << bits) < n) ++bits;
        size_t tb = cl.sort_tmp_bytes;
        e = hipcub::DeviceRadixSort::SortPairs(p.sort_tmp, tb, d->col, p.keys_out, p.perm_in, p.perm_out, (int)nnz, 0,
                                               bits, st);
        if (e != hipSuccess) return set_error(GLRM_EHIP, "radix sort: %s", hipGetErrorString(e));
        hipLaunchKernelGGL(gather_csc_kernel, dim3(nblk(nnz)), dim3(256), 0, st, p.perm_out, d->row, d->A, nnz,
                           p.csc_row, p.csc_val);
    }
    hipLaunchKernelGGL(seg_ptr_kernel, dim3(nblk(n + 1)), dim3(256), 0, st, p.keys_out, nnz, n, p.col_ptr);
    hipLaunchKernelGGL(seg_count_kernel, dim3(nblk(n)), dim3(256), 0, st, p.col_ptr, n, col_count);
    if ((e = hipGetLastError()) != hipSuccess) return set_error(GLRM_EHIP, "COO set-up launch: %s", hipGetErrorString(e));
    return GLRM_OK;
}

int coo_check_result(const CooLayout &cl, char *base, hipStream_t st)
{
    int32_t f = 0;
    CooPtrs p = ptrs(cl, base);
    if (hipMemcpyAsync(&f, p.flags, sizeof f, hipMemcpyDeviceToHost, st) != hipSuccess) return 1;
    if (hipStreamSynchronize(st) != hipSuccess) return 1;
    return f;
}

// ---- the walks ----------------------------------------------------------------

// Sum over a group of L consecutive lanes (L = 4, 8 or 16) with DPP moves;
// every lane of the group gets a sum, the group's first lane always in the
// same order.
template <int L>
__device__ __forceinline__ float group_sum(float v)
{
    static_assert(L == 4 || L == 8 || L == 16, "entry groups of 4, 8 or 16 lanes");
    if constexpr (L == 16) v += dpp_mov<0x128>(v);   // row_ror:8
    if constexpr (L >= 8) v += dpp_mov<0x141>(v);    // row_half_mirror: 7 - (l mod 8)
    v += dpp_mov<0x4E>(v);                           // quad_perm [2,3,0,1]
    v += dpp_mov<0xB1>(v);                           // quad_perm [1,0,3,2]
    return v;
}

template <int L>
__device__ __forceinline__ double group_sum64(double v)
{
#pragma unroll
    for (int o = L / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the entry groups of a wavefront (lanes with the same q).
template <int L>
__device__ __forceinline__ float across_groups(float v)
{
#pragma unroll
    for (int o = L; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float dot4(const float4 &a, const float4 &b)
{
    return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
}

struct WalkArgs {
    int64_t rows;            // rows of the walked view (m for the row walk, n for the column walk)
    int32_t k;
    const int32_t *ptr;      // rows + 1
    const int32_t *idx;      // nnz: index into the other factor
    const float *val;        // nnz
    const uint8_t *codes;    // per column of A
    bool codes_by_entry;     // row walk: code of idx[e]; column walk: code of the walked row
    LossTab lt;
    Reg reg;
    float *U;                // walked factor, rows x k (user layout)
    float *Us;               // walked factor, rows x kp (padded)
    const float *Vs;         // other factor, padded
    float *alpha;
    float step_up, step_down;
    float *dU;               // gradient output (lossgrad mode)
    double *part_obj;        // per wave: objective part (lossgrad) / decided row objectives (step)
    int32_t *part_rej;       // per wave: rejected rows (step)
    bool reg_only;           // step: accumulate only r of the decided rows (the other walk counts the loss)
};

// One entry's loss (and derivative) in the walk.  LK >= 0: every column has
// loss kind LK (compile time); LK < 0: the code of the entry's column.
// wcol: the entry's column of A (its loss weight, when the table has weights).
template <int LK>
__device__ __forceinline__ void walk_lg(const WalkArgs &a, int code, int wcol, float z, float v, float &l, float &g)
{
    if constexpr (LK >= 0) {
        loss_lg_k<LK>(a.lt.levels[0], a.lt.param[0], z, v, l, g);
    } else {
        const int q = a.lt.uniform >= 0 ? a.lt.uniform : code;
        loss_lg(a.lt.kind[q], a.lt.levels[q], a.lt.param[q], z, v, l, g);
        if (a.lt.colw) {
            const float w = a.lt.colw[wcol];
            l *= w;
            g *= w;
        }
    }
}

template <int LK>
__device__ __forceinline__ float walk_l(const WalkArgs &a, int code, int wcol, float z, float v)
{
    if constexpr (LK >= 0) {
        return loss_l_k<LK>(a.lt.levels[0], a.lt.param[0], z, v);
    } else {
        const int q = a.lt.uniform >= 0 ? a.lt.uniform : code;
        const float l = loss_l(a.lt.kind[q], a.lt.levels[q], a.lt.param[q], z, v);
        return a.lt.colw ? l * a.lt.colw[wcol] : l;
    }
}

// MODE 0: loss (+ gradient if dU); MODE 1: full half-step; MODE 2: loss in double.
// The walk goes through a row's entries in chunks of NS * E: every lane first
// loads the indices and values of its NS entries, then issues their NS factor
// gathers, and only then reduces, so each chunk costs two memory round trips.
template <int KP, int MODE, int LK>
__global__ __launch_bounds__(256) void walk_kernel(WalkArgs a)
{
    constexpr int L = KP / 4;       // lanes per entry
    constexpr int E = 64 / L;       // entries per wavefront step
    constexpr int NS = 8;           // steps per chunk
    const int lane = threadIdx.x & 63;
    const int slot = lane / L, q = lane % L;
    const int64_t wave = (int64_t)blockIdx.x * CW + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * CW;
    double wsum = 0.0;
    int wrej = 0;
    const float4 *V4 = reinterpret_cast<const float4 *>(a.Vs);
    for (int64_t i = wave; i < a.rows; i += nwaves) {
        const int32_t beg = a.ptr[i], end = a.ptr[i + 1];
        const float4 x = reinterpret_cast<const float4 *>(a.Us + i * KP)[q];
        const int rowcode = a.codes_by_entry ? 0 : a.codes[i];
        if constexpr (MODE == 2) {
            double acc = 0.0;
            for (int32_t b = beg; b < end; b += NS * E) {
                int32_t j[NS];
                float v[NS];
                float4 y[NS];
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int32_t e = b + s * E + slot;
                    j[s] = e < end ? a.idx[e] : -1;
                    v[s] = e < end ? a.val[e] : 0.0f;
                }
#pragma unroll
                for (int s = 0; s < NS; ++s) y[s] = j[s] >= 0 ? V4[(int64_t)j[s] * L + q] : float4{0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    double z = (double)x.x * y[s].x + (double)x.y * y[s].y + (double)x.z * y[s].z +
                               (double)x.w * y[s].w;
                    z = group_sum64<L>(z);
                    if (j[s] >= 0 && q == 0) {
                        const int code = a.codes_by_entry ? a.codes[j[s]] : rowcode;
                        const int qq = a.lt.uniform >= 0 ? a.lt.uniform : code;
                        const double wv = a.lt.colw ? (double)a.lt.colw[a.codes_by_entry ? j[s] : (int)i] : 1.0;
                        acc += wv * loss_l64(a.lt.kind[qq], a.lt.levels[qq], (double)a.lt.param[qq], z, (double)v[s]);
                    }
                }
            }
            wsum += acc;
            continue;
        }
        float f = 0.0f;
        float4 gacc = {0.f, 0.f, 0.f, 0.f};
        for (int32_t b = beg; b < end; b += NS * E) {
            int32_t j[NS];
            float v[NS];
            float4 y[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int32_t e = b + s * E + slot;
                j[s] = e < end ? a.idx[e] : -1;
                v[s] = e < end ? a.val[e] : 0.0f;
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) y[s] = j[s] >= 0 ? V4[(int64_t)j[s] * L + q] : float4{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const float z = group_sum<L>(dot4(x, y[s]));
                float l = 0.f, gr = 0.f;
                if (j[s] >= 0)
                    walk_lg<LK>(a, a.codes_by_entry ? a.codes[j[s]] : rowcode, a.codes_by_entry ? j[s] : (int)i, z,
                                v[s], l, gr);
                if (q == 0) f += l;
                gacc.x += gr * y[s].x; gacc.y += gr * y[s].y; gacc.z += gr * y[s].z; gacc.w += gr * y[s].w;
            }
        }
        gacc.x = across_groups<L>(gacc.x);
        gacc.y = across_groups<L>(gacc.y);
        gacc.z = across_groups<L>(gacc.z);
        gacc.w = across_groups<L>(gacc.w);
        f = across_groups<L>(group_sum<L>(f));   // only q == 0 lanes were nonzero
        if constexpr (MODE == 0) {
            wsum += (double)f;
            if (a.dU && slot == 0) {
                const float gv[4] = {gacc.x, gacc.y, gacc.z, gacc.w};
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    if (4 * q + s < a.k) a.dU[i * a.k + 4 * q + s] = gv[s];
            }
        } else {
            const float al = a.alpha[i];
            const float xv[4] = {x.x, x.y, x.z, x.w};
            const float gv[4] = {gacc.x, gacc.y, gacc.z, gacc.w};
            float xp[4];
            float rc = 0.f, rcp = 0.f;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bool in = 4 * q + s < a.k;
                xp[s] = in ? prox_elem(a.reg, al, xv[s] - al * gv[s], 4 * q + s) : 0.0f;
                rc += in ? reg_elem(a.reg, xv[s], 4 * q + s) : 0.0f;
                rcp += in ? reg_elem_trial(a.reg, xp[s], 4 * q + s) : 0.0f;
            }
            rc = group_sum<L>(rc);
            rcp = group_sum<L>(rcp);
            const float4 xp4 = {xp[0], xp[1], xp[2], xp[3]};
            float fp = 0.0f;
            for (int32_t b = beg; b < end; b += NS * E) {
                int32_t j[NS];
                float v[NS];
                float4 y[NS];
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int32_t e = b + s * E + slot;
                    j[s] = e < end ? a.idx[e] : -1;
                    v[s] = e < end ? a.val[e] : 0.0f;
                }
#pragma unroll
                for (int s = 0; s < NS; ++s) y[s] = j[s] >= 0 ? V4[(int64_t)j[s] * L + q] : float4{0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const float z = group_sum<L>(dot4(xp4, y[s]));
                    if (j[s] >= 0 && q == 0)
                        fp += walk_l<LK>(a, a.codes_by_entry ? a.codes[j[s]] : rowcode, a.codes_by_entry ? j[s] : (int)i,
                                         z, v[s]);
                }
            }
            fp = across_groups<L>(group_sum<L>(fp));
            const float F0 = f + rc, F1 = fp + rcp;
            const bool acc = F1 <= F0;
            if (acc && slot == 0) {
                reinterpret_cast<float4 *>(a.Us + i * KP)[q] = xp4;
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    if (4 * q + s < a.k) a.U[i * a.k + 4 * q + s] = xp[s];
            }
            if (lane == 0) {
                a.alpha[i] = acc ? al * a.step_up : al * a.step_down;
                if (a.reg_only) wsum += acc ? (double)rcp : (double)rc;
                else wsum += acc ? (double)F1 : (double)F0;
                wrej += acc ? 0 : 1;
            }
        }
    }
    if constexpr (MODE == 2) wsum = sum_lanes64<64>(wsum);  // lanes with q == 0 hold the parts
    if (lane == 0) {
        a.part_obj[wave] = wsum;
        if (MODE == 1) a.part_rej[wave] = wrej;
    }
}

// Sum of decided objectives of the columns + the row regularizers of X^t.
__global__ __launch_bounds__(256) void coo_finalize_kernel(const double *colF, const int32_t *colrej, int ncol,
                                                           const double *rowreg, const int32_t *rowrej, int nrow,
                                                           double *stats, long long *istats, double *history,
                                                           int sweep)
{
    __shared__ double sF[256];
    __shared__ long long sr[256], sc[256];
    double F = 0.0;
    long long rr = 0, rc = 0;
    for (int q = threadIdx.x; q < ncol; q += 256) { F += colF[q]; rc += colrej[q]; }
    for (int q = threadIdx.x; q < nrow; q += 256) { F += rowreg[q]; rr += rowrej[q]; }
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
        stats[0] = sF[0];
        istats[0] = sr[0];
        istats[1] = sc[0];
        if (history) history[sweep] = sF[0];
    }
}

// ---- host side ----------------------------------------------------------------

static int walk_grid(int64_t rows)
{
    const int64_t blocks = (rows + CW - 1) / CW;
    return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, COO_MAX_WAVES / CW));
}

template <int MODE, int LK>
static hipError_t launch_walk_lk(const WalkArgs &a, int kp, int grid, hipStream_t st)
{
    switch (kp) {
    case 16: hipLaunchKernelGGL((walk_kernel<16, MODE, LK>), dim3(grid), dim3(256), 0, st, a); break;
    case 32: hipLaunchKernelGGL((walk_kernel<32, MODE, LK>), dim3(grid), dim3(256), 0, st, a); break;
    case 64: hipLaunchKernelGGL((walk_kernel<64, MODE, LK>), dim3(grid), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// A table with the quadratic loss everywhere gets its own instances.
template <int MODE>
static hipError_t launch_walk(const WalkArgs &a, int kp, int grid, hipStream_t st)
{
    if (MODE != 2 && a.lt.uniform >= 0 && a.lt.kind[a.lt.uniform] == L_QUAD) {
        WalkArgs b = a;
        b.lt.levels[0] = a.lt.levels[a.lt.uniform];
        b.lt.param[0] = a.lt.param[a.lt.uniform];
        return launch_walk_lk<MODE, L_QUAD>(b, kp, grid, st);
    }
    return launch_walk_lk<MODE, -1>(a, kp, grid, st);
}

static WalkArgs row_walk(const glrm_data *d, const CooPtrs &p, const uint8_t *codes, const LossTab &lt)
{
    WalkArgs a;
    memset(&a, 0, sizeof a);
    a.rows = d->m; a.k = d->k;
    a.ptr = p.row_ptr; a.idx = d->col; a.val = d->A;
    a.codes = codes; a.codes_by_entry = true;
    a.lt = lt;
    a.Us = p.xs; a.Vs = p.ys;
    return a;
}

static WalkArgs col_walk(const glrm_data *d, const CooPtrs &p, const uint8_t *codes, const LossTab &lt)
{
    WalkArgs a;
    memset(&a, 0, sizeof a);
    a.rows = d->n; a.k = d->k;
    a.ptr = p.col_ptr; a.idx = p.csc_row; a.val = p.csc_val;
    a.codes = codes; a.codes_by_entry = false;
    a.lt = lt;
    a.Us = p.ys; a.Vs = p.xs;
    return a;
}

static int pad_factors(const glrm_data *d, int kp, const CooPtrs &p, const float *X, const float *Y, hipStream_t st)
{
    hipLaunchKernelGGL(pad_factor_kernel, dim3(nblk(d->m * kp)), dim3(256), 0, st, X, d->m, d->k, kp, p.xs);
    hipLaunchKernelGGL(pad_factor_kernel, dim3(nblk(d->n * kp)), dim3(256), 0, st, Y, d->n, d->k, kp, p.ys);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GLRM_OK : set_error(GLRM_EHIP, "pad factors: %s", hipGetErrorString(e));
}

static int coo_prec_ok(int prec)
{
    if (prec == GLRM_FP32 || prec == GLRM_FP64) return GLRM_OK;
    return set_error(GLRM_EUNSUPPORTED, "the COO layout computes in FP32 (and FP64 for the objective); "
                     "bfloat16 precisions are built for the dense layout only");
}

int coo_objective(const glrm_data *d, const CooLayout &cl, char *base, const uint8_t *codes, const LossTab &lt,
                  const float *X, const float *Y, int prec, double **parts, int *nparts, hipStream_t st)
{
    if (int rc = coo_prec_ok(prec)) return rc;
    CooPtrs p = ptrs(cl, base);
    int rc = pad_factors(d, cl.kp, p, X, Y, st);
    if (rc) return rc;
    WalkArgs a = row_walk(d, p, codes, lt);
    a.part_obj = p.partA;
    const int grid = walk_grid(d->m);
    hipError_t e = prec == GLRM_FP64 ? launch_walk<2>(a, cl.kp, grid, st) : launch_walk<0>(a, cl.kp, grid, st);
    if (e != hipSuccess) return set_error(GLRM_EHIP, "COO objective: %s", hipGetErrorString(e));
    *parts = p.partA;
    *nparts = grid * CW;
    return GLRM_OK;
}

int coo_grad(const glrm_data *d, int kp, const CooLayout &cl, char *base, const uint8_t *codes, const LossTab &lt,
             const float *X, const float *Y, int prec, float *dX, float *dY, double **parts, int *nparts,
             hipStream_t st)
{
    if (int rc0 = coo_prec_ok(prec)) return rc0;
    CooPtrs p = ptrs(cl, base);
    int rc = pad_factors(d, kp, p, X, Y, st);
    if (rc) return rc;
    WalkArgs a = row_walk(d, p, codes, lt);
    a.dU = dX;
    a.part_obj = p.partA;
    const int grid = walk_grid(d->m);
    hipError_t e = launch_walk<0>(a, kp, grid, st);
    if (e != hipSuccess) return set_error(GLRM_EHIP, "COO gradient (rows): %s", hipGetErrorString(e));
    WalkArgs b = col_walk(d, p, codes, lt);
    b.dU = dY;
    b.part_obj = p.partB;
    e = launch_walk<0>(b, kp, walk_grid(d->n), st);
    if (e != hipSuccess) return set_error(GLRM_EHIP, "COO gradient (columns): %s", hipGetErrorString(e));
    *parts = p.partA;
    *nparts = grid * CW;
    return GLRM_OK;
}

int coo_fit_supported(const glrm_data *d, int kp, const CooLayout &cl, int prec)
{
    (void)d; (void)kp; (void)cl;
    return coo_prec_ok(prec);
}

int coo_fit(const glrm_data *d, int kp, const CooLayout &cl, char *base, const uint8_t *codes, const LossTab &lt,
            float *X, float *Y, float *alpha_x, float *alpha_y, const glrm_fit_opts *o, double *history,
            double *stats, long long *istats, int *sweeps, hipStream_t st,
            const std::function<hipError_t(int)> &tstart, const std::function<hipError_t()> &tstop)
{
    CooPtrs p = ptrs(cl, base);
    int rc = pad_factors(d, kp, p, X, Y, st);
    if (rc) return rc;
    WalkArgs ra = row_walk(d, p, codes, lt);
    ra.reg = Reg{d->rx.kind, d->rx.weight, d->offset ? 1 : 0};
    ra.U = X; ra.alpha = alpha_x; ra.step_up = o->step_up; ra.step_down = o->step_down;
    ra.part_obj = p.partA; ra.part_rej = p.ipartA; ra.reg_only = true;
    WalkArgs ca = col_walk(d, p, codes, lt);
    ca.reg = Reg{d->ry.kind, d->ry.weight, d->offset ? 2 : 0};
    ca.U = Y; ca.alpha = alpha_y; ca.step_up = o->step_up; ca.step_down = o->step_down;
    ca.part_obj = p.partB; ca.part_rej = p.ipartB;
    const int grid_r = walk_grid(d->m), grid_c = walk_grid(d->n);
    double F_prev = NAN;
    *sweeps = 0;
    for (int t = 0; t < o->max_sweeps; ++t) {
        hipError_t e = tstart(0);
        if (e == hipSuccess) e = launch_walk<1>(ra, kp, grid_r, st);
        if (e == hipSuccess) e = tstop();
        if (e == hipSuccess) e = tstart(1);
        if (e == hipSuccess) e = launch_walk<1>(ca, kp, grid_c, st);
        if (e == hipSuccess) e = tstop();
        if (e == hipSuccess) e = tstart(3);
        if (e != hipSuccess) return set_error(GLRM_EHIP, "COO sweep: %s", hipGetErrorString(e));
        // F = decided column objectives (loss + rt) + r of the decided rows
        hipLaunchKernelGGL(coo_finalize_kernel, dim3(1), dim3(256), 0, st, p.partB, p.ipartB, grid_c * CW, p.partA,
                           p.ipartA, grid_r * CW, stats, istats, history, t);
        if ((e = tstop()) != hipSuccess) return set_error(GLRM_EHIP, "COO timing: %s", hipGetErrorString(e));
        if ((e = hipGetLastError()) != hipSuccess) return set_error(GLRM_EHIP, "COO finalize: %s", hipGetErrorString(e));
        *sweeps = t + 1;
        if (o->tol > 0.0) {
            double F;
            if (hipMemcpyAsync(&F, stats, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return set_error(GLRM_EHIP, "COO fit: reading the objective failed");
            if (t > 0 && (F_prev - F) <= o->tol * std::fabs(F_prev)) break;
            F_prev = F;
        }
    }
    return GLRM_OK;
}

}  // namespace glrm
