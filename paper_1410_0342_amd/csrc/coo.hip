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
// The row-blocked column step: NX partial sets (one per XCD: workgroup w
// runs on XCD w mod 8 and takes the row blocks rb = w mod 8 (mod 8)), each
// wave owning at most CB_JW(kp) columns, CB_GMIN..CB_GMAX workgroups per XCD,
// and row blocks of about 1 MB of the padded float32 X.
constexpr int NX = 8;
#ifndef GLRM_CB_NS
#define GLRM_CB_NS 4
#endif
#ifndef GLRM_CB_GMIN
#define GLRM_CB_GMIN 128
#endif
constexpr int CB_NS = GLRM_CB_NS;
constexpr int CB_GMIN = GLRM_CB_GMIN, CB_GMAX = 256;
constexpr int64_t CB_MAX_SEGMENTS = int64_t(1) << 28;
static int cb_jw_max(int kp) { return kp == 64 ? 32 : 64; }
#ifndef GLRM_CB_RB_ADJ
#define GLRM_CB_RB_ADJ 0
#endif
static int cb_rb_shift(int kp) { return (kp == 16 ? 14 : (kp == 32 ? 13 : 12)) - GLRM_CB_RB_ADJ; }
static int bits_for(int64_t v)
{
    int b = 1;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

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
    hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (const int *)nullptr, (int *)nullptr, (const int *)nullptr,
                                       (int *)nullptr, (int)nnz, 0, bits_for(d->n), (hipStream_t)0);
    // the row-blocked copy
    cl.rb_shift = cb_rb_shift(kp);
    cl.nb = (d->m + (int64_t(1) << cl.rb_shift) - 1) >> cl.rb_shift;
    const int64_t nseg = cl.nb * d->n;
    // packed entries: column in 16 bits
    cl.blk = d->nnz > 0 && nseg < CB_MAX_SEGMENTS && d->n <= std::min<int64_t>(65536, (int64_t)cb_jw_max(kp) * CW * CB_GMAX);
    if (cl.blk) {
        size_t tb2 = 0;
        hipcub::DeviceRadixSort::SortPairs(nullptr, tb2, (const int *)nullptr, (int *)nullptr, (const int *)nullptr,
                                           (int *)nullptr, (int)nnz, 0, bits_for(nseg), (hipStream_t)0);
        tb = std::max(tb, tb2);
    }
    cl.sort_tmp_bytes = tb;
    cl.sort_tmp = take(tb);
    if (cl.blk) {
        cl.bkey = take(sizeof(int32_t) * nnz);
        cl.bperm = take(sizeof(int32_t) * nnz);
        cl.brow = take(sizeof(int32_t) * nnz);
        cl.bval = take(sizeof(float) * nnz);
        cl.seg = take(sizeof(int32_t) * (nseg + 1));
        cl.bpart0 = take(sizeof(float) * NX * d->n * (kp + 1));
        cl.bpart1 = take(sizeof(float) * NX * d->n);
        cl.yplus = take(sizeof(float) * d->n * kp);
        cl.hold = take(sizeof(float) * d->n);
        cl.rplus = take(sizeof(float) * d->n);
    }
    cl.flags = take(sizeof(int32_t) * 4);
    cl.part_bytes = (sizeof(double) * 2 + sizeof(int32_t) * 2) * COO_MAX_WAVES;
    cl.part = take(cl.part_bytes);
    cl.xs = take(sizeof(float) * d->m * kp);
    cl.ys = take(sizeof(float) * d->n * kp);
    cl.xsb = take(2 * d->m * kp);
    cl.ysb = take(2 * d->n * kp);
    if (cl.blk) cl.zc = take(sizeof(float) * nnz);
}

struct CooPtrs {
    int32_t *row_ptr, *col_ptr, *csc_row, *perm_in, *perm_out, *keys_out, *flags;
    float *csc_val, *xs, *ys, *zc;
    __bf16 *xsb, *ysb;
    int32_t *bkey, *bperm, *brow, *seg;
    float *bval, *bpart0, *bpart1, *yplus, *hold, *rplus;
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
    p.xsb = (__bf16 *)(b + cl.xsb);
    p.ysb = (__bf16 *)(b + cl.ysb);
    p.zc = (float *)(b + cl.zc);
    p.bkey = (int32_t *)(b + cl.bkey);
    p.bperm = (int32_t *)(b + cl.bperm);
    p.brow = (int32_t *)(b + cl.brow);
    p.bval = (float *)(b + cl.bval);
    p.seg = (int32_t *)(b + cl.seg);
    p.bpart0 = (float *)(b + cl.bpart0);
    p.bpart1 = (float *)(b + cl.bpart1);
    p.yplus = (float *)(b + cl.yplus);
    p.hold = (float *)(b + cl.hold);
    p.rplus = (float *)(b + cl.rplus);
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

// The row-blocked copy: value and packed (column << 16 | row within its block).
__global__ void gather_blk_kernel(const int32_t *perm, const int32_t *row, const int32_t *col, const float *val,
                                  int64_t nnz, int shift, uint32_t *packed, float *bval)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < nnz) {
        const int32_t e = perm[p];
        packed[p] = ((uint32_t)col[e] << 16) | ((uint32_t)row[e] & ((1u << shift) - 1));
        bval[p] = val[e];
    }
}

// Key of an entry in the row-blocked order: (row block, column).
__global__ void blk_key_kernel(const int32_t *row, const int32_t *col, int64_t nnz, int64_t n, int shift, int32_t *key)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < nnz) key[e] = (int32_t)((int64_t)(row[e] >> shift) * n + col[e]);
}

// Padded copies of a factor: dst (rows x kp) from src (rows x k), and its
// bfloat16 rounding (round to nearest even).
__global__ void pad_factor_kernel(const float *src, int64_t rows, int32_t k, int32_t kp, float *dst, __bf16 *dstb)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= rows * kp) return;
    const int64_t i = t / kp;
    const int c = (int)(t % kp);
    const float v = c < k ? src[i * k + c] : 0.0f;
    dst[t] = v;
    dstb[t] = (__bf16)v;
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
    if (cl.blk) {
        // (row block, column) keys of the row-sorted list; a stable sort keeps
        // each segment's rows in order
        const int64_t nseg = cl.nb * n;
        hipLaunchKernelGGL(blk_key_kernel, dim3(nblk(nnz)), dim3(256), 0, st, d->row, d->col, nnz, n, cl.rb_shift,
                           p.bkey);
        size_t tb = cl.sort_tmp_bytes;
        e = hipcub::DeviceRadixSort::SortPairs(p.sort_tmp, tb, p.bkey, p.keys_out, p.perm_in, p.bperm, (int)nnz, 0,
                                               bits_for(nseg), st);
        if (e != hipSuccess) return set_error(GLRM_EHIP, "radix sort (row blocks): %s", hipGetErrorString(e));
        hipLaunchKernelGGL(gather_blk_kernel, dim3(nblk(nnz)), dim3(256), 0, st, p.bperm, d->row, d->col, d->A, nnz,
                           cl.rb_shift, reinterpret_cast<uint32_t *>(p.brow), p.bval);
        hipLaunchKernelGGL(seg_ptr_kernel, dim3(nblk(nseg + 1)), dim3(256), 0, st, p.keys_out, nnz, nseg, p.seg);
    }
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

// A lane's C consecutive coordinates of a factor row (C = 4 or 8).
template <int C>
struct Part {
    float4 v[C / 4];
};

template <int KP, int C>
__device__ __forceinline__ Part<C> load_part(const float4 *__restrict__ F4, int64_t row, int q)
{
    Part<C> r;
#pragma unroll
    for (int u = 0; u < C / 4; ++u) r.v[u] = F4[row * (KP / 4) + q * (C / 4) + u];
    return r;
}

template <int C>
__device__ __forceinline__ float dot_part(const Part<C> &a, const Part<C> &b)
{
    float s = dot4(a.v[0], b.v[0]);
#pragma unroll
    for (int u = 1; u < C / 4; ++u) s += dot4(a.v[u], b.v[u]);
    return s;
}

template <int C>
__device__ __forceinline__ void axpy_part(Part<C> &acc, float g, const Part<C> &x)
{
#pragma unroll
    for (int u = 0; u < C / 4; ++u) {
        acc.v[u].x += g * x.v[u].x; acc.v[u].y += g * x.v[u].y;
        acc.v[u].z += g * x.v[u].z; acc.v[u].w += g * x.v[u].w;
    }
}

// The bfloat16 copy of a lane's C coordinates (C / 2 packed pairs).
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2_t;
typedef __attribute__((ext_vector_type(2))) float f32x2_t;

template <int C>
struct PartB {
    uint32_t w[C / 2];
};

template <int KP, int C>
__device__ __forceinline__ PartB<C> load_partb(const __bf16 *__restrict__ F, int64_t row, int q)
{
    PartB<C> r;
    const uint32_t *p = reinterpret_cast<const uint32_t *>(F + row * KP + (int64_t)q * C);
    if constexpr (C == 8) {
        const uint4 u = *reinterpret_cast<const uint4 *>(p);
        r.w[0] = u.x; r.w[1] = u.y; r.w[2] = u.z; r.w[3] = u.w;
    } else {
        const uint2 u = *reinterpret_cast<const uint2 *>(p);
        r.w[0] = u.x; r.w[1] = u.y;
    }
    return r;
}

// A step d in bfloat16 pairs (round to nearest even).
template <int C>
__device__ __forceinline__ PartB<C> to_partb(const Part<C> &d)
{
    PartB<C> r;
#pragma unroll
    for (int u = 0; u < C / 4; ++u) {
        const bf16x2_t a = __builtin_convertvector((f32x2_t){d.v[u].x, d.v[u].y}, bf16x2_t);
        const bf16x2_t b = __builtin_convertvector((f32x2_t){d.v[u].z, d.v[u].w}, bf16x2_t);
        r.w[2 * u] = __builtin_bit_cast(uint32_t, a);
        r.w[2 * u + 1] = __builtin_bit_cast(uint32_t, b);
    }
    return r;
}

// sum over the lane's coordinates of d_c v_c, both in bfloat16, float32 sums
template <int C>
__device__ __forceinline__ float dot_partb(const PartB<C> &d, const PartB<C> &v)
{
    float s = 0.0f;
#pragma unroll
    for (int p = 0; p < C / 2; ++p)
        s = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, d.w[p]), __builtin_bit_cast(bf16x2_t, v.w[p]),
                                            s, false);
    return s;
}

template <int C>
__device__ __forceinline__ Part<C> sub_part(const Part<C> &a, const Part<C> &b)
{
    Part<C> r;
#pragma unroll
    for (int u = 0; u < C / 4; ++u)
        r.v[u] = float4{a.v[u].x - b.v[u].x, a.v[u].y - b.v[u].y, a.v[u].z - b.v[u].z, a.v[u].w - b.v[u].w};
    return r;
}

template <int KP, int C>
__device__ __forceinline__ void store_partb(__bf16 *F, int64_t row, int q, const Part<C> &x)
{
    const PartB<C> b = to_partb<C>(x);
    uint32_t *p = reinterpret_cast<uint32_t *>(F + row * KP + (int64_t)q * C);
#pragma unroll
    for (int t = 0; t < C / 2; ++t) p[t] = b.w[t];
}

// Coordinates per lane in the row-blocked column passes: 8 (groups of KP / 8
// lanes per entry, fewer lanes repeating the loss and the butterfly), 4 at
// KP = 16.
template <int KP>
constexpr int cb_c() { return KP == 16 ? 4 : 8; }

// Indices and values of the chunk at b of a segment [first, end): entries
// b + s E + slot for the steps s the chunk has (a uniform early exit; the
// caller runs exactly as many).  An entry past the segment's end repeats the
// segment's first one, so every load and gather stays in bounds, and the
// caller masks it out.
// O32: byte offsets of the entries fit 32 bits (checked on the host), so each
// load takes the array's base in scalar registers and one 32-bit vector
// offset instead of a 64-bit address per lane.
template <int NS, int E, typename T, bool O32 = false>
__device__ __forceinline__ void chunk_load(const T *__restrict__ idx, const float *__restrict__ val, int32_t b,
                                           int32_t end, int32_t first, int slot, T (&i)[NS], float (&v)[NS])
{
    static_assert(sizeof(T) == sizeof(float), "one 32-bit word per entry");
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (b + s * E >= end) break;
        const int32_t e = b + s * E + slot;
        const int32_t ee = e < end ? e : first;
        if constexpr (O32) {
            const uint32_t off = (uint32_t)ee * 4u;
            i[s] = *reinterpret_cast<const T *>(reinterpret_cast<const char *>(idx) + off);
            v[s] = *reinterpret_cast<const float *>(reinterpret_cast<const char *>(val) + off);
        } else {
            i[s] = idx[ee];
            v[s] = val[ee];
        }
    }
}

// A gathered factor row (the lane's C coordinates of row `row` of a padded
// rows x KP factor).  O32: the row's byte offset fits 32 bits (checked on the
// host), as for chunk_load.
template <int KP, int C, bool O32>
__device__ __forceinline__ Part<C> gather_part(const float *__restrict__ F, int32_t row, int q)
{
    if constexpr (O32) {
        const float4 *p = reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(F) +
                                                           ((uint32_t)row * KP + (uint32_t)(q * C)) * 4u);
        Part<C> r;
#pragma unroll
        for (int u = 0; u < C / 4; ++u) r.v[u] = p[u];
        return r;
    } else {
        return load_part<KP, C>(reinterpret_cast<const float4 *>(F), row, q);
    }
}

template <int KP, int C, bool O32>
__device__ __forceinline__ PartB<C> gather_partb(const __bf16 *__restrict__ F, int32_t row, int q)
{
    if constexpr (O32) {
        const char *p = reinterpret_cast<const char *>(F) + ((uint32_t)row * KP + (uint32_t)(q * C)) * 2u;
        PartB<C> r;
        if constexpr (C == 8) {
            const uint4 u = *reinterpret_cast<const uint4 *>(p);
            r.w[0] = u.x; r.w[1] = u.y; r.w[2] = u.z; r.w[3] = u.w;
        } else {
            const uint2 u = *reinterpret_cast<const uint2 *>(p);
            r.w[0] = u.x; r.w[1] = u.y;
        }
        return r;
    } else {
        return load_partb<KP, C>(F, row, q);
    }
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
    // the bfloat16 trial (MODE 3): bf16 copies of both padded factors
    const __bf16 *Vsb;
    __bf16 *Usb;
    int64_t nnz;             // entries of the walked view
    int64_t vrows;           // rows of the gathered factor Vs (and Vsb)
};

// The bfloat16 trial keeps a row's products z_ij in LDS between the two
// passes when the row has at most ZMAX entries.
constexpr int ZMAX = 512;

// One entry's loss (and derivative) in the walk.  LK >= 0: every column has
// loss kind LK (compile time); LK < 0: the code of the entry's column.
// wcol: the entry's column of A (its loss weight, when the table has weights).
template <int LK>
__device__ __forceinline__ void walk_lg(const LossTab &lt, int code, int wcol, float z, float v, float &l, float &g)
{
    if constexpr (LK >= 0) {
        loss_lg_k<LK>(lt.levels[0], lt.param[0], z, v, l, g);
    } else {
        const int q = lt.uniform >= 0 ? lt.uniform : code;
        loss_lg(lt.kind[q], lt.levels[q], lt.param[q], z, v, l, g);
        if (lt.colw) {
            const float w = lt.colw[wcol];
            l *= w;
            g *= w;
        }
    }
}

template <int LK>
__device__ __forceinline__ float walk_l(const LossTab &lt, int code, int wcol, float z, float v)
{
    if constexpr (LK >= 0) {
        return loss_l_k<LK>(lt.levels[0], lt.param[0], z, v);
    } else {
        const int q = lt.uniform >= 0 ? lt.uniform : code;
        const float l = loss_l(lt.kind[q], lt.levels[q], lt.param[q], z, v);
        return lt.colw ? l * lt.colw[wcol] : l;
    }
}

// MODE 0: loss (+ gradient if dU); MODE 1: full half-step; MODE 2: loss in
// double; MODE 3: the half-step with the bfloat16 trial: the first pass keeps
// every z_ij = x_i . y_j, and the trial products are z_ij + (x+ - x) . y_j with
// the step and y_j in bfloat16 (two coordinates per dot2 instruction), so the
// second pass gathers half the bytes.  A wave owns one row at a time; groups of L = KP / C lanes share an entry,
// each lane holding C coordinates, so a factor row is one coalesced gather
// and z = x_i . y_j a short butterfly over the group.  The walk goes through
// a row's entries in chunks of up to NS steps of E entries: every lane first
// loads the indices and values of its entries, then issues their factor
// gathers, and only then reduces (a row's last chunk runs only the steps it
// has; entries past the row's end repeat its first entry and are masked).
template <int KP, int MODE, int LK, bool O32>
__global__ __launch_bounds__(256) void walk_kernel(WalkArgs a)
{
    constexpr int C = cb_c<KP>(), L = KP / C, E = 64 / L, NS = CB_NS;
    const int lane = threadIdx.x & 63;
    const int slot = lane / L, q = lane % L;
    const int64_t wave = (int64_t)blockIdx.x * CW + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * CW;
    double wsum = 0.0;
    int wrej = 0;
    const float4 *U4 = reinterpret_cast<const float4 *>(a.Us);
    auto code_of = [&](int32_t j, int rowcode) { return a.codes_by_entry ? (int)a.codes[j] : rowcode; };
    constexpr bool BT = MODE == 3;
    __shared__ float zbuf[BT ? CW : 1][BT ? ZMAX : 1];
    float *zrow = zbuf[BT ? (threadIdx.x >> 6) : 0];
    for (int64_t i = wave; i < a.rows; i += nwaves) {
        const int32_t beg = a.ptr[i], end = a.ptr[i + 1];
        const Part<C> x = load_part<KP, C>(U4, i, q);
        const int rowcode = a.codes_by_entry ? 0 : a.codes[i];
        if constexpr (MODE == 2) {
            double acc = 0.0;
            for (int32_t b = beg; b < end; b += NS * E) {
                int32_t j[NS];
                float v[NS];
                Part<C> y[NS];
                chunk_load<NS, E, int32_t, O32>(a.idx, a.val, b, end, beg, slot, j, v);
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (b + s * E >= end) break;
                    y[s] = gather_part<KP, C, O32>(a.Vs, j[s], q);
                }
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (b + s * E >= end) break;
                    double z = 0.0;
#pragma unroll
                    for (int u = 0; u < C / 4; ++u)
                        z += (double)x.v[u].x * y[s].v[u].x + (double)x.v[u].y * y[s].v[u].y +
                             (double)x.v[u].z * y[s].v[u].z + (double)x.v[u].w * y[s].v[u].w;
                    z = group_sum64<L>(z);
                    if (b + s * E + slot < end && q == 0) {
                        const int qq = a.lt.uniform >= 0 ? a.lt.uniform : code_of(j[s], rowcode);
                        const double wv = a.lt.colw ? (double)a.lt.colw[a.codes_by_entry ? j[s] : (int)i] : 1.0;
                        acc += wv * loss_l64(a.lt.kind[qq], a.lt.levels[qq], (double)a.lt.param[qq], z, (double)v[s]);
                    }
                }
            }
            wsum += acc;
            continue;
        }
        float f = 0.0f;
        Part<C> gacc = {};
        const bool keep_z = BT && end - beg <= ZMAX;
        for (int32_t b = beg; b < end; b += NS * E) {
            int32_t j[NS];
            float v[NS];
            Part<C> y[NS];
            chunk_load<NS, E, int32_t, O32>(a.idx, a.val, b, end, beg, slot, j, v);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (b + s * E >= end) break;
                y[s] = gather_part<KP, C, O32>(a.Vs, j[s], q);
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (b + s * E >= end) break;
                const bool ok = b + s * E + slot < end;
                const float z = group_sum<L>(dot_part<C>(x, y[s]));
                if (BT && keep_z && ok && q == 0) zrow[b - beg + s * E + slot] = z;
                float l, gr;
                walk_lg<LK>(a.lt, code_of(j[s], rowcode), a.codes_by_entry ? j[s] : (int)i, z, v[s], l, gr);
                f += (ok && q == 0) ? l : 0.0f;
                axpy_part<C>(gacc, ok ? gr : 0.0f, y[s]);
            }
        }
#pragma unroll
        for (int u = 0; u < C / 4; ++u) {
            gacc.v[u].x = across_groups<L>(gacc.v[u].x);
            gacc.v[u].y = across_groups<L>(gacc.v[u].y);
            gacc.v[u].z = across_groups<L>(gacc.v[u].z);
            gacc.v[u].w = across_groups<L>(gacc.v[u].w);
        }
        f = across_groups<L>(group_sum<L>(f));   // only q == 0 lanes were nonzero
        if constexpr (MODE == 0) {
            wsum += (double)f;
            if (a.dU && slot == 0) {
#pragma unroll
                for (int u = 0; u < C / 4; ++u) {
                    const float gv[4] = {gacc.v[u].x, gacc.v[u].y, gacc.v[u].z, gacc.v[u].w};
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int c = C * q + 4 * u + t;
                        if (c < a.k) a.dU[i * a.k + c] = gv[t];
                    }
                }
            }
        } else {
            const float al = a.alpha[i];
            Part<C> xp;
            float rc = 0.f, rcp = 0.f;
#pragma unroll
            for (int u = 0; u < C / 4; ++u) {
                const float xv[4] = {x.v[u].x, x.v[u].y, x.v[u].z, x.v[u].w};
                const float gv[4] = {gacc.v[u].x, gacc.v[u].y, gacc.v[u].z, gacc.v[u].w};
                float pv[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int c = C * q + 4 * u + t;
                    const bool in = c < a.k;
                    pv[t] = in ? prox_elem(a.reg, al, xv[t] - al * gv[t], c) : 0.0f;
                    rc += in ? reg_elem(a.reg, xv[t], c) : 0.0f;
                    rcp += in ? reg_elem_trial(a.reg, pv[t], c) : 0.0f;
                }
                xp.v[u] = float4{pv[0], pv[1], pv[2], pv[3]};
            }
            rc = group_sum<L>(rc);
            rcp = group_sum<L>(rcp);
            float fp = 0.0f;
            if (BT && keep_z) {
                // z held in LDS (written by lanes q == 0 of each group, read by all of it)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const PartB<C> db = to_partb<C>(sub_part<C>(xp, x));
                const __bf16 *Vb = a.Vsb;
                for (int32_t b = beg; b < end; b += NS * E) {
                    int32_t j[NS];
                    float v[NS];
                    PartB<C> yb[NS];
                    chunk_load<NS, E, int32_t, O32>(a.idx, a.val, b, end, beg, slot, j, v);
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        if (b + s * E >= end) break;
                        yb[s] = gather_partb<KP, C, O32>(Vb, j[s], q);
                    }
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        if (b + s * E >= end) break;
                        const int32_t e = b - beg + s * E + slot;
                        const bool ok = e < end - beg;
                        const float z0 = zrow[ok ? e : 0];
                        const float z = z0 + group_sum<L>(dot_partb<C>(db, yb[s]));
                        const float l = walk_l<LK>(a.lt, code_of(j[s], rowcode), a.codes_by_entry ? j[s] : (int)i, z, v[s]);
                        fp += (ok && q == 0) ? l : 0.0f;
                    }
                }
                // the next row's products may not overwrite these before every lane has read them
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            } else
            for (int32_t b = beg; b < end; b += NS * E) {
                int32_t j[NS];
                float v[NS];
                Part<C> y[NS];
                chunk_load<NS, E, int32_t, O32>(a.idx, a.val, b, end, beg, slot, j, v);
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (b + s * E >= end) break;
                    y[s] = gather_part<KP, C, O32>(a.Vs, j[s], q);
                }
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (b + s * E >= end) break;
                    const bool ok = b + s * E + slot < end;
                    const float z = group_sum<L>(dot_part<C>(xp, y[s]));
                    const float l = walk_l<LK>(a.lt, code_of(j[s], rowcode), a.codes_by_entry ? j[s] : (int)i, z, v[s]);
                    fp += (ok && q == 0) ? l : 0.0f;
                }
            }
            fp = across_groups<L>(group_sum<L>(fp));
            const float F0 = f + rc, F1 = fp + rcp;
            const bool acc = F1 <= F0;
            if (acc && slot == 0) {
                if constexpr (BT) store_partb<KP, C>(a.Usb, i, q, xp);
#pragma unroll
                for (int u = 0; u < C / 4; ++u) {
                    reinterpret_cast<float4 *>(a.Us + i * KP)[q * (C / 4) + u] = xp.v[u];
                    const float pv[4] = {xp.v[u].x, xp.v[u].y, xp.v[u].z, xp.v[u].w};
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int c = C * q + 4 * u + t;
                        if (c < a.k) a.U[i * a.k + c] = pv[t];
                    }
                }
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
        if (MODE == 1 || MODE == 3) a.part_rej[wave] = wrej;
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

// ---- the column step on the row-blocked copy ----------------------------------
//
// A column's entries sit in segments, one per row block.  The workgroups of
// one XCD take that XCD's row blocks in order and, within a block, every
// wave the segments of its own columns, so all waves of an XCD gather x_i
// from the same ~1 MB block of X at about the same time: the gathers hit the
// XCD's L2 instead of going out to memory.  A wave accumulates its columns
// across row blocks in LDS (each lane only its own slots) and writes one
// partial per column and XCD; the NX partials are summed in a fixed order.
struct ColBlkArgs {
    int64_t n, nb;
    int32_t k, jw;          // jw: columns per wave at most (wave w owns w, w + V, ...)
    int32_t rb_shift;       // rows per block: 2^rb_shift
    const int32_t *seg;     // nb * n + 1 segment pointers
    const uint32_t *row;    // nnz, row-blocked order: column << 16 | row within its block
    const float *val;
    const uint8_t *codes;   // per column of A
    LossTab lt;
    const float *Xs;        // m x kp
    const float *Ys;        // n x kp: y (passes 0, 2) or the trial y+ (passes 1, 3)
    float *part;            // passes 0, 2: NX x n x (kp + 1) (gradient, loss); 1, 3: NX x n (trial loss)
    // the bfloat16 trial: pass 2 keeps z of every entry (row-blocked order),
    // pass 3 forms z + (y+ - y) . x_i from it with the bf16 copy of X
    float *zc;
    const __bf16 *Xsb;
    const float *Ycur;      // n x kp: y (pass 3)
};

// PASS 0: loss-part gradient and loss of every column at Ys; PASS 1: loss at Ys.
// PASS 2: PASS 0 that also keeps every entry's z; PASS 3: PASS 1 from those z
// and the bfloat16 copy of X (the bf16 trial).
// Per row block a wave first reads its segments' pointers (one per lane),
// then walks its segments as one stream of chunks of up to NS * E entries
// (a segment's last chunk runs only the steps it has), the indices and
// values of the next chunk loading while the current chunk's rows are
// gathered and used.  A segment's sums go into its column's LDS slots
// (lane groups reduced first; each lane adds only its own slots).
template <int KP, int PASS, int LK>
__global__ __launch_bounds__(256) void colblk_kernel(ColBlkArgs a)
{
    constexpr int C = cb_c<KP>(), L = KP / C, E = 64 / L, NS = CB_NS;
    constexpr bool GRAD = PASS == 0 || PASS == 2, BT = PASS == 3;
    constexpr int W = GRAD ? KP + 1 : 1;
    extern __shared__ float cb_lds[];
    const int lane = threadIdx.x & 63, slot = lane / L, q = lane % L;
    const int xcd = (int)(blockIdx.x % NX);
    const int64_t V = (int64_t)(gridDim.x / NX) * CW;
    const int64_t wv = (int64_t)(blockIdx.x / NX) * CW + (threadIdx.x >> 6);
    float *acc = cb_lds + (size_t)(threadIdx.x >> 6) * a.jw * W;
    const bool owner = GRAD ? slot == 0 : lane == 0;     // lanes holding accumulator slots
    for (int jl = 0; jl < a.jw; ++jl) {
        if (GRAD && owner) {
#pragma unroll
            for (int t = 0; t < C; ++t) acc[jl * W + C * q + t] = 0.0f;
        }
        if (lane == 0) acc[jl * W + W - 1] = 0.0f;
    }
    // columns of this wave: j = wv + jl * V, jl < jc (<= 64, one per lane)
    const int jc = wv < a.n ? (int)((a.n - wv + V - 1) / V) : 0;
    const float4 *Y4 = reinterpret_cast<const float4 *>(a.Ys);
    const uint32_t rmask = (1u << a.rb_shift) - 1;
    for (int64_t rb = xcd; rb < a.nb; rb += NX) {
        int32_t pb = 0, pe = 0;
        if (lane < jc) {
            const int64_t o = rb * a.n + wv + (int64_t)lane * V;
            pb = a.seg[o];
            pe = a.seg[o + 1];
        }
        const int64_t rbase = rb << a.rb_shift;
        // the first non-empty segment at or after jl
        auto next_seg = [&](int jl) {
            while (jl < jc && __builtin_amdgcn_readlane(pb, jl) == __builtin_amdgcn_readlane(pe, jl)) ++jl;
            return jl;
        };
        int jl = next_seg(0);
        if (jl >= jc) continue;
        int32_t first = __builtin_amdgcn_readlane(pb, jl), b = first, end = __builtin_amdgcn_readlane(pe, jl);
        uint32_t i[NS];
        float v[NS], zv[NS];
        auto load_c = [&](int32_t b0, int32_t e0, int32_t f0, uint32_t (&ii)[NS], float (&vv)[NS], float (&zz)[NS]) {
            chunk_load<NS, E>(a.row, a.val, b0, e0, f0, slot, ii, vv);
            if constexpr (BT) chunk_load<NS, E>(a.row, a.zc, b0, e0, f0, slot, ii, zz);
        };
        load_c(b, end, first, i, v, zv);
        Part<C> y = load_part<KP, C>(Y4, wv + (int64_t)jl * V, q);
        // the step of the column (bf16 trial)
        PartB<C> db = {};
        if constexpr (BT) db = to_partb<C>(sub_part<C>(y, load_part<KP, C>(reinterpret_cast<const float4 *>(a.Ycur), wv + (int64_t)jl * V, q)));
        float f = 0.0f;
        Part<C> g = {};
        while (true) {
            Part<C> x[NS];
            PartB<C> xb[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (b + s * E >= end) break;
                // within the row block (a row below 2^16 of it): 32-bit offsets from the block's base
                if constexpr (BT) xb[s] = gather_partb<KP, C, true>(a.Xsb + rbase * KP, (int32_t)(i[s] & rmask), q);
                else x[s] = gather_part<KP, C, true>(a.Xs + rbase * KP, (int32_t)(i[s] & rmask), q);
            }
            // the next chunk: the rest of this segment, else the next non-empty one
            int jl2 = jl;
            int32_t b2 = b + NS * E, end2 = end, first2 = first;
            if (b2 >= end) {
                jl2 = next_seg(jl + 1);
                if (jl2 < jc) {
                    b2 = first2 = __builtin_amdgcn_readlane(pb, jl2);
                    end2 = __builtin_amdgcn_readlane(pe, jl2);
                }
            }
            uint32_t i2[NS];
            float v2[NS], zv2[NS];
            Part<C> y2 = y;
            PartB<C> db2 = db;
            if (jl2 < jc) {
                load_c(b2, end2, first2, i2, v2, zv2);
                if (jl2 != jl) {
                    y2 = load_part<KP, C>(Y4, wv + (int64_t)jl2 * V, q);
                    if constexpr (BT)
                        db2 = to_partb<C>(sub_part<C>(
                            y2, load_part<KP, C>(reinterpret_cast<const float4 *>(a.Ycur), wv + (int64_t)jl2 * V, q)));
                }
            }
            const int64_t j = wv + (int64_t)jl * V;
            const int code = a.codes[j];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (b + s * E >= end) break;
                const bool ok = b + s * E + slot < end;
                if constexpr (BT) {
                    const float z = zv[s] + group_sum<L>(dot_partb<C>(db, xb[s]));
                    const float l = walk_l<LK>(a.lt, code, (int)j, z, v[s]);
                    f += (ok && q == 0) ? l : 0.0f;
                    continue;
                }
                const float z = group_sum<L>(dot_part<C>(x[s], y));
                if constexpr (PASS == 2) {
                    if (ok && q == 0) a.zc[b + s * E + slot] = z;
                }
                if constexpr (GRAD) {
                    float l, gr;
                    walk_lg<LK>(a.lt, code, (int)j, z, v[s], l, gr);
                    f += (ok && q == 0) ? l : 0.0f;
                    axpy_part<C>(g, ok ? gr : 0.0f, x[s]);
                } else {
                    const float l = walk_l<LK>(a.lt, code, (int)j, z, v[s]);
                    f += (ok && q == 0) ? l : 0.0f;
                }
            }
            if (jl2 != jl) {
                // the segment is done: into the column's accumulator
                f = across_groups<L>(group_sum<L>(f));   // only q == 0 lanes were nonzero
                if constexpr (GRAD) {
#pragma unroll
                    for (int u = 0; u < C / 4; ++u) {
                        float4 &gv = g.v[u];
                        gv.x = across_groups<L>(gv.x);
                        gv.y = across_groups<L>(gv.y);
                        gv.z = across_groups<L>(gv.z);
                        gv.w = across_groups<L>(gv.w);
                        if (owner) {
                            float *d = acc + jl * W + C * q + 4 * u;
                            d[0] += gv.x; d[1] += gv.y; d[2] += gv.z; d[3] += gv.w;
                        }
                    }
                    g = Part<C>{};
                }
                if (lane == 0) acc[jl * W + W - 1] += f;
                f = 0.0f;
            }
            if (jl2 >= jc) break;
            jl = jl2;
            b = b2;
            end = end2;
            first = first2;
            y = y2;
            db = db2;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                i[s] = i2[s];
                v[s] = v2[s];
                zv[s] = zv2[s];
            }
        }
    }
    int jl = 0;
    for (int64_t j = wv; j < a.n; j += V, ++jl) {
        float *dst = a.part + ((int64_t)xcd * a.n + j) * W;
        if (GRAD && owner) {
#pragma unroll
            for (int t = 0; t < C; ++t) dst[C * q + t] = acc[jl * W + C * q + t];
        }
        if (lane == 0) dst[W - 1] = acc[jl * W + W - 1];
    }
}

struct ColStepArgs {
    int64_t n;
    int32_t k;
    const float *part0;     // NX x n x (kp + 1)
    const float *part1;     // NX x n
    const float *Yin;       // n x k (current columns)
    float *alpha;
    Reg reg;
    float step_up, step_down;
    float *yplus;           // n x kp: the trial columns
    float *hold, *rplus;    // n: objective of the current column (loss + rt), rt of the trial column
    float *dY;              // gradient mode: n x k output (then no step is taken)
    float *Y;               // decide: n x k, updated
    float *ys;              // decide: n x kp padded copy, updated
    __bf16 *ysb;            // decide: its bfloat16 copy, updated
    double *partF;          // decide: per block, decided column objectives
    int32_t *partR;         // decide: per block, rejected columns
};

// The sum of the NX partials (fixed order), then either the gradient out
// (dY) or the proximal gradient step of every column: the trial y+, the
// current column's objective and rt(y+).
template <int KP>
__global__ __launch_bounds__(256) void colblk_step_kernel(ColStepArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = t / KP;
    const int c = (int)(t % KP);
    const bool valid = j < a.n;
    float g = 0.0f, fo = 0.0f;
    if (valid) {
#pragma unroll
        for (int x = 0; x < NX; ++x) g += a.part0[((int64_t)x * a.n + j) * (KP + 1) + c];
        if (c == 0) {
#pragma unroll
            for (int x = 0; x < NX; ++x) fo += a.part0[((int64_t)x * a.n + j) * (KP + 1) + KP];
        }
    }
    if (a.dY) {
        if (valid && c < a.k) a.dY[j * a.k + c] = g;
        return;
    }
    float y = 0.0f, al = 0.0f;
    if (valid) {
        al = a.alpha[j];
        if (c < a.k) y = a.Yin[j * a.k + c];
    }
    const bool in = valid && c < a.k;
    const float yp = in ? prox_elem(a.reg, al, y - al * g, c) : 0.0f;
    float ro = in ? reg_elem(a.reg, y, c) : 0.0f;
    float rp = in ? reg_elem_trial(a.reg, yp, c) : 0.0f;
    ro = sum_lanes<KP>(ro);
    rp = sum_lanes<KP>(rp);
    if (valid) {
        a.yplus[j * KP + c] = yp;
        if (c == 0) {
            a.hold[j] = fo + ro;
            a.rplus[j] = rp;
        }
    }
}

// The step rule of every column: the trial objective (NX partials in a fixed
// order + rt(y+)) against the current one; accepted columns take y+.
template <int KP>
__global__ __launch_bounds__(256) void colblk_decide_kernel(ColStepArgs a)
{
    __shared__ double s_F[4];
    __shared__ int s_r[4];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = t / KP;
    const int c = (int)(t % KP);
    const bool valid = j < a.n;
    float fp = 0.0f;
    if (valid && c == 0) {
#pragma unroll
        for (int x = 0; x < NX; ++x) fp += a.part1[(int64_t)x * a.n + j];
    }
    fp = sum_lanes<KP>(fp);   // the same value in every lane of the column
    double Fj = 0.0;
    int rj = 0;
    if (valid) {
        fp += a.rplus[j];
        const float ho = a.hold[j];
        const bool acc = fp <= ho;
        if (acc) {
            const float yp = a.yplus[j * KP + c];
            a.ys[j * KP + c] = yp;
            a.ysb[j * KP + c] = (__bf16)yp;
            if (c < a.k) a.Y[j * a.k + c] = yp;
        }
        if (c == 0) {
            const float al = a.alpha[j];
            a.alpha[j] = acc ? al * a.step_up : al * a.step_down;
            Fj = acc ? (double)fp : (double)ho;
            rj = acc ? 0 : 1;
        }
    }
    Fj = sum_lanes64<64>(Fj);
    rj = (int)sum_lanes<64>((float)rj);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { s_F[w] = Fj; s_r[w] = rj; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.partF[blockIdx.x] = s_F[0] + s_F[1] + s_F[2] + s_F[3];
        a.partR[blockIdx.x] = s_r[0] + s_r[1] + s_r[2] + s_r[3];
    }
}

// ---- host side ----------------------------------------------------------------

static int walk_grid(int64_t rows)
{
    const int64_t blocks = (rows + CW - 1) / CW;
    return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, COO_MAX_WAVES / CW));
}

template <int MODE, int LK, bool O32>
static hipError_t launch_walk_o(const WalkArgs &a, int kp, int grid, hipStream_t st)
{
    switch (kp) {
    case 16: hipLaunchKernelGGL((walk_kernel<16, MODE, LK, O32>), dim3(grid), dim3(256), 0, st, a); break;
    case 32: hipLaunchKernelGGL((walk_kernel<32, MODE, LK, O32>), dim3(grid), dim3(256), 0, st, a); break;
    case 64: hipLaunchKernelGGL((walk_kernel<64, MODE, LK, O32>), dim3(grid), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// 32-bit byte offsets when every entry's offset (nnz * 4 bytes of indices,
// as of values) and every gathered row's (vrows * kp floats) fit 32 bits;
// the FP64 objective keeps the 64-bit form.
static bool walk_offsets_fit_32(const WalkArgs &a, int kp)
{
    const int64_t lim = (int64_t)1 << 32;
    return a.nnz * 4 <= lim && a.vrows * kp * 4 <= lim;
}

template <int MODE, int LK>
static hipError_t launch_walk_lk(const WalkArgs &a, int kp, int grid, hipStream_t st)
{
    if constexpr (MODE != 2) {
        if (walk_offsets_fit_32(a, kp)) return launch_walk_o<MODE, LK, true>(a, kp, grid, st);
    }
    return launch_walk_o<MODE, LK, false>(a, kp, grid, st);
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
    a.nnz = d->nnz; a.vrows = d->n;
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
    a.nnz = d->nnz; a.vrows = d->m;
    return a;
}

// Launch shape of the row-blocked column passes: workgroups per XCD and the
// columns each wave owns.
struct ColBlkShape {
    int g, jw;
};

static ColBlkShape colblk_shape(int64_t n, int kp)
{
    const int64_t need = (n + (int64_t)cb_jw_max(kp) * CW - 1) / ((int64_t)cb_jw_max(kp) * CW);
    const int g = (int)std::min<int64_t>(CB_GMAX, std::max<int64_t>(CB_GMIN, need));
    const int jw = (int)std::max<int64_t>(1, (n + (int64_t)g * CW - 1) / ((int64_t)g * CW));
    return ColBlkShape{g, jw};
}

template <int PASS, int LK>
static hipError_t launch_colblk_lk(const ColBlkArgs &a, int kp, const ColBlkShape &sh, hipStream_t st)
{
    const size_t lds = sizeof(float) * CW * sh.jw * (PASS == 0 || PASS == 2 ? kp + 1 : 1);
    const dim3 grid((unsigned)(NX * sh.g));
    switch (kp) {
    case 16: hipLaunchKernelGGL((colblk_kernel<16, PASS, LK>), grid, dim3(256), lds, st, a); break;
    case 32: hipLaunchKernelGGL((colblk_kernel<32, PASS, LK>), grid, dim3(256), lds, st, a); break;
    case 64: hipLaunchKernelGGL((colblk_kernel<64, PASS, LK>), grid, dim3(256), lds, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int PASS>
static hipError_t launch_colblk(const ColBlkArgs &a, int kp, const ColBlkShape &sh, hipStream_t st)
{
    if (a.lt.uniform >= 0 && a.lt.kind[a.lt.uniform] == L_QUAD) {
        ColBlkArgs b = a;
        b.lt.levels[0] = a.lt.levels[a.lt.uniform];
        b.lt.param[0] = a.lt.param[a.lt.uniform];
        return launch_colblk_lk<PASS, L_QUAD>(b, kp, sh, st);
    }
    return launch_colblk_lk<PASS, -1>(a, kp, sh, st);
}

template <int DECIDE>
static hipError_t launch_colstep(const ColStepArgs &a, int kp, hipStream_t st)
{
    const dim3 grid(nblk(a.n * kp));
    switch (kp) {
    case 16:
        if (DECIDE) hipLaunchKernelGGL(colblk_decide_kernel<16>, grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL(colblk_step_kernel<16>, grid, dim3(256), 0, st, a);
        break;
    case 32:
        if (DECIDE) hipLaunchKernelGGL(colblk_decide_kernel<32>, grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL(colblk_step_kernel<32>, grid, dim3(256), 0, st, a);
        break;
    case 64:
        if (DECIDE) hipLaunchKernelGGL(colblk_decide_kernel<64>, grid, dim3(256), 0, st, a);
        else hipLaunchKernelGGL(colblk_step_kernel<64>, grid, dim3(256), 0, st, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static ColBlkArgs colblk_args(const glrm_data *d, const CooLayout &cl, const CooPtrs &p, const uint8_t *codes,
                              const LossTab &lt, int kp)
{
    ColBlkArgs a;
    memset(&a, 0, sizeof a);
    a.n = d->n; a.nb = cl.nb; a.k = d->k;
    a.jw = colblk_shape(d->n, kp).jw;
    a.seg = p.seg; a.row = reinterpret_cast<const uint32_t *>(p.brow); a.val = p.bval;
    a.rb_shift = cl.rb_shift;
    a.codes = codes; a.lt = lt;
    a.Xs = p.xs;
    return a;
}

static int pad_factors(const glrm_data *d, int kp, const CooPtrs &p, const float *X, const float *Y, hipStream_t st)
{
    hipLaunchKernelGGL(pad_factor_kernel, dim3(nblk(d->m * kp)), dim3(256), 0, st, X, d->m, d->k, kp, p.xs, p.xsb);
    hipLaunchKernelGGL(pad_factor_kernel, dim3(nblk(d->n * kp)), dim3(256), 0, st, Y, d->n, d->k, kp, p.ys, p.ysb);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GLRM_OK : set_error(GLRM_EHIP, "pad factors: %s", hipGetErrorString(e));
}

// The COO layout's precisions: FP32; FP64 for the objective; BF16, whose
// trial passes take z + (x+ - x) . y with the step and the gathered factor
// in bfloat16 (objective and gradient calls compute as FP32).
static int coo_prec_ok(int prec)
{
    if (prec == GLRM_FP32 || prec == GLRM_FP64 || prec == GLRM_BF16) return GLRM_OK;
    return set_error(GLRM_EUNSUPPORTED, "the COO layout computes in FP32 or BF16 (and FP64 for the objective); "
                     "BF16_PLAIN is built for the dense layout only");
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
    hipError_t e = prec == GLRM_FP64 ? launch_walk<2>(a, cl.kp, grid, st) : launch_walk<0>(a, cl.kp, grid, st);  // BF16: as FP32
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
    if (cl.blk) {
        ColBlkArgs b = colblk_args(d, cl, p, codes, lt, kp);
        b.Ys = p.ys;
        b.part = p.bpart0;
        e = launch_colblk<0>(b, kp, colblk_shape(d->n, kp), st);
        ColStepArgs s;
        memset(&s, 0, sizeof s);
        s.n = d->n; s.k = d->k; s.part0 = p.bpart0; s.dY = dY;
        if (e == hipSuccess) e = launch_colstep<0>(s, kp, st);
    } else {
        WalkArgs b = col_walk(d, p, codes, lt);
        b.dU = dY;
        b.part_obj = p.partB;
        e = launch_walk<0>(b, kp, walk_grid(d->n), st);
    }
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
    ra.Vsb = p.ysb; ra.Usb = p.xsb;
    WalkArgs ca = col_walk(d, p, codes, lt);
    ca.reg = Reg{d->ry.kind, d->ry.weight, d->offset ? 2 : 0};
    ca.U = Y; ca.alpha = alpha_y; ca.step_up = o->step_up; ca.step_down = o->step_down;
    ca.part_obj = p.partB; ca.part_rej = p.ipartB;
    ca.Vsb = p.xsb; ca.Usb = p.ysb;
    const bool bt = o->precision == GLRM_BF16;   // the bfloat16 trial passes
    const int grid_r = walk_grid(d->m), grid_c = walk_grid(d->n);
    // the row-blocked column step: gradient pass, step, trial pass, decision
    const ColBlkShape sh = colblk_shape(d->n, kp);
    ColBlkArgs c0, c1;
    ColStepArgs cs;
    memset(&cs, 0, sizeof cs);
    if (cl.blk) {
        c0 = colblk_args(d, cl, p, codes, lt, kp);
        c0.Ys = p.ys; c0.part = p.bpart0;
        c0.zc = p.zc; c0.Xsb = p.xsb; c0.Ycur = p.ys;
        c1 = c0;
        c1.Ys = p.yplus; c1.part = p.bpart1;
        cs.n = d->n; cs.k = d->k; cs.part0 = p.bpart0; cs.part1 = p.bpart1;
        cs.Yin = Y; cs.alpha = alpha_y; cs.reg = ca.reg; cs.step_up = o->step_up; cs.step_down = o->step_down;
        cs.yplus = p.yplus; cs.hold = p.hold; cs.rplus = p.rplus;
        cs.Y = Y; cs.ys = p.ys; cs.ysb = p.ysb; cs.partF = p.partB; cs.partR = p.ipartB;
    }
    const int ncolparts = cl.blk ? (int)nblk(d->n * kp) : grid_c * CW;
    double F_prev = NAN;
    *sweeps = 0;
    for (int t = 0; t < o->max_sweeps; ++t) {
        hipError_t e = tstart(0);
        if (e == hipSuccess) e = bt ? launch_walk<3>(ra, kp, grid_r, st) : launch_walk<1>(ra, kp, grid_r, st);
        if (e == hipSuccess) e = tstop();
        if (e == hipSuccess) e = tstart(1);
        if (cl.blk) {
            if (e == hipSuccess) e = bt ? launch_colblk<2>(c0, kp, sh, st) : launch_colblk<0>(c0, kp, sh, st);
            if (e == hipSuccess) e = launch_colstep<0>(cs, kp, st);
            if (e == hipSuccess) e = bt ? launch_colblk<3>(c1, kp, sh, st) : launch_colblk<1>(c1, kp, sh, st);
            if (e == hipSuccess) e = launch_colstep<1>(cs, kp, st);
        } else {
            if (e == hipSuccess) e = bt ? launch_walk<3>(ca, kp, grid_c, st) : launch_walk<1>(ca, kp, grid_c, st);
        }
        if (e == hipSuccess) e = tstop();
        if (e == hipSuccess) e = tstart(3);
        if (e != hipSuccess) return set_error(GLRM_EHIP, "COO sweep: %s", hipGetErrorString(e));
        // F = decided column objectives (loss + rt) + r of the decided rows
        hipLaunchKernelGGL(coo_finalize_kernel, dim3(1), dim3(256), 0, st, p.partB, p.ipartB, ncolparts, p.partA,
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
