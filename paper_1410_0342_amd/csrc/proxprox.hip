// The prox-prox update for quadratic losses (Sections 7.2, 7.3), dense layout.
// See proxprox.h.  Per half-step: a Gram pass over the table (the dense
// contraction, on the matrix cores), a solve pass (one wavefront per row: Cholesky of
// G_i + I / (2 alpha) in double in LDS, then `inner` prox-prox updates by
// triangular solves), and a check pass (old and trial row objectives summed
// from the table, the step rule of Section 7.2).  Every sum has a fixed order.
#include <algorithm>
#include <utility>

#include "glrm_kernels.h"
#include "proxprox.h"

namespace glrm {

static unsigned nblk(int64_t n, int per = 256) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

template <int KP>
constexpr int PP_NT = KP / 4;                         // 4 x 4 tiles a side
template <int KP>
constexpr int PP_UT = PP_NT<KP> * (PP_NT<KP> + 1) / 2;  // upper tiles
// One row's Gram data: the upper tiles, padded to four per wavefront of the
// Gram pass (its stores then take no branch), then b in four 16-wide slots.
template <int KP>
constexpr int PP_TW = (PP_UT<KP> + 3) / 4;            // upper tiles per wavefront of the Gram pass
template <int KP>
constexpr int PP_BOFF = 4 * PP_TW<KP> * 16;           // offset of b
template <int KP>
constexpr int PP_GSZ = PP_BOFF<KP> + 64;              // floats of one row's Gram data

int pp_gram_floats(int kp)
{
    switch (kp) {
    case 16: return PP_GSZ<16>;
    case 32: return PP_GSZ<32>;
    default: return PP_GSZ<64>;
    }
}

// The Gram data keeps only the upper 4 x 4 tiles that meet the rank: tile
// rows and columns 0 .. nt - 1 with nt = ceil(k / 4), in the order of the
// upper triangle's rows (slot u of `nt (nt + 1) / 2`).
__device__ __forceinline__ int pp_nt(int k) { return (k + 3) / 4; }

// slot u -> (ta, tb), ta <= tb, for nt tile rows (runtime)
__device__ __forceinline__ void tile_of_rt(int u, int nt, int &ta, int &tb)
{
    ta = tb = -1;
    for (int r = 0; r < nt; ++r) {
        const int len = nt - r;
        if (u < len) {
            ta = r;
            tb = r + u;
            return;
        }
        u -= len;
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

// One 64-column chunk of a panel pass in registers: the fixed factor's 64
// rows, the panel's 16 x 64 entries (NaN past the rows and columns) and the
// column weights.  A chunk is loaded while the previous one computes, then
// stored into LDS.
template <int KP>
struct PPChunk {
    static constexpr int CH = 64, NV = CH * KP / 256, NE = 16 * CH / 256;
    float v[NV], e[NE], w;

    __device__ __forceinline__ void load(const PPArgs &a, int64_t i0, int64_t j0, int64_t c1)
    {
        const int t = threadIdx.x;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const int f = t + 256 * q, jj = f / KP, c = f % KP;
            const int64_t j = j0 + jj;
            v[q] = (j < c1 && c < a.k) ? a.V[j * a.k + c] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int f = t + 256 * q, rr = f / CH, jj = f % CH;
            const int64_t ii = i0 + rr, j = j0 + jj;
            e[q] = (ii < a.rows && j < c1) ? a.T[ii * a.ldt + j] : __builtin_nanf("");
        }
        const int64_t j = j0 + (t & (CH - 1));
        w = (a.wcol && j < c1) ? a.wcol[j] : 1.0f;
    }

    __device__ __forceinline__ void store(float (*sV)[KP + 4], float (*sT)[CH + 4], float *sW) const
    {
        const int t = threadIdx.x;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const int f = t + 256 * q;
            sV[f / KP][f % KP] = v[q];
        }
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int f = t + 256 * q;
            sT[f / CH][f % CH] = e[q];
        }
        if (t < CH) sW[t] = w;
    }
};

// ---- Gram pass --------------------------------------------------------------------
// On the matrix cores: for a 16-row panel, G(16 rows x 16 pairs) += M(16 x 4) .
// W(4 x 16) with M_ij the entry's weight (0 where A_ij is unobserved) and
// W_j[(a, b)] = v_ja v_jb over the sixteen pairs of one upper 4 x 4 tile of
// G; b(16 rows x 16 coordinates) += (M o A)(16 x 4) . V(4 x 16).  The fp32
// 16x16x4 product keeps the products and sums in fp32, as the solve needs.
// Wavefront w owns the slots u = w, w + 4, ... of the tiles that meet the
// rank (TW of them, the instance chosen for k) and the b tile w.
// Columns go in chunks of 64 staged in LDS: the panel's 16 x 64 entries and
// the chunk's rows of the fixed factor.
template <int KP, int TW>
__global__ __launch_bounds__(256) void pp_gram_kernel(PPArgs a)
{
    constexpr int GSZ = PP_GSZ<KP>, BOFF = PP_BOFF<KP>;
    static_assert(4 * TW <= 4 * PP_TW<KP>, "slots");
    static_assert(KP / 16 <= 4, "one b tile per wavefront");
    constexpr int CH = 64;                    // staged columns
    __shared__ float sV[CH][KP + 4];
    __shared__ float sT[16][CH + 4];
    __shared__ float sW[CH];
    // w as a scalar: the tile tests below are then scalar branches, not exec-mask ones
    const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int li = lane & 15, g = lane >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * 16;
    const int64_t per = (a.cols + a.splits - 1) / a.splits;
    const int64_t c0 = (int64_t)blockIdx.y * per, c1 = min<int64_t>(a.cols, c0 + per);
    const int k = a.k;
    // this lane's coordinates of each of its upper tiles (a = 4 ta + li / 4, b = 4 tb + li % 4)
    const int nt = pp_nt(k), ut = nt * (nt + 1) / 2;
    int ca[TW], cb[TW];
    bool act[TW];
#pragma unroll
    for (int q = 0; q < TW; ++q) {
        const int u = w + 4 * q;
        int ta = -1, tb = -1;
        if (u < ut) tile_of_rt(u, nt, ta, tb);
        act[q] = u < ut;
        ca[q] = act[q] ? 4 * ta + (li >> 2) : 0;
        cb[q] = act[q] ? 4 * tb + (li & 3) : 0;
    }
    f32x4 acc[TW], bacc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < TW; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bool bact = w < KP / 16 && 16 * w < k;   // this wavefront's b tile: coordinates 16 w ..
    const int bcol = bact ? 16 * w + li : li;        // (an inactive tile reads column li, never stored)
    const float wr = (a.wrow && i0 + li < a.rows) ? a.wrow[i0 + li] : 1.0f;
    // where the panel's rows go (chosen here, away from the products' results)
    const int64_t rowsp = (a.rows + 15) / 16 * 16;
    float *const obase = a.splits > 1 ? a.gpart + (int64_t)blockIdx.y * rowsp * GSZ : a.gram;
    PPChunk<KP> chunk;
    if (c0 < c1) chunk.load(a, i0, c0, c1);
    for (int64_t j0 = c0; j0 < c1; j0 += CH) {
        __syncthreads();
        chunk.store(sV, sT, sW);
        __syncthreads();
        if (j0 + CH < c1) chunk.load(a, i0, j0 + CH, c1);   // in flight while this chunk computes
        const int nks = (int)((min<int64_t>(CH, c1 - j0) + 3) / 4);
#pragma unroll 4
        for (int ks = 0; ks < nks; ++ks) {
            const int jj = 4 * ks + g;              // this lane's column of the step (k index g)
            const float av = sT[li][jj];            // row li (A operand: row li, k g)
            const float sw = sW[jj];
            const bool obs = av == av;
            const float m = obs ? wr * sw : 0.0f;
            const float mb = obs ? m * av : 0.0f;
            // Every slot's product runs, inactive ones on coordinates 0 (never
            // stored): a branch per slot made the compiler move the
            // accumulators between register files around each product.
#pragma unroll
            for (int q = 0; q < TW; ++q) {
                const float bv = sV[jj][ca[q]] * sV[jj][cb[q]];     // B operand: k g, column li
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bv, acc[q], 0, 0, 0);
            }
            bacc = __builtin_amdgcn_mfma_f32_16x16x4f32(mb, sV[jj][bcol], bacc, 0, 0, 0);
        }
    }
    // One more product into every accumulator, so that the reads below follow
    // a product in straight-line code: the wait states the reads need are then
    // the compiler's straight-line ones, not counted across the loop's exit
    // branch.  Every store below is unconditional (the output holds padded
    // rows and padded tile slots).
#pragma unroll
    for (int q = 0; q < TW; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(0.0f, 0.0f, acc[q], 0, 0, 0);
    bacc = __builtin_amdgcn_mfma_f32_16x16x4f32(0.0f, 0.0f, bacc, 0, 0, 0);
    // lane (li, g) holds rows 4 g + r of column li of each tile
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + 4 * g + r;          // < rowsp
        float *out = obase + i * GSZ;
#pragma unroll
        for (int q = 0; q < TW; ++q) out[(w + 4 * q) * 16 + li] = act[q] ? acc[q][r] : 0.0f;
        out[BOFF + 16 * w + li] = bact ? bacc[r] : 0.0f;
    }
}

// out[e] = sum over the np partial sets (each `stride` floats apart) of part[e], in order.
__global__ void pp_reduce_kernel(const float *part, int32_t np, int64_t len, int64_t stride, float *out)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= len) return;
    float s = 0.0f;
    for (int p = 0; p < np; ++p) s += part[(int64_t)p * stride + e];
    out[e] = s;
}

// Slots per wavefront of the Gram pass for rank k: the smallest instance
// that holds ceil(nt (nt + 1) / 2 / 4) of them.
template <int KP, int... TWS>
static hipError_t pp_gram_launch(const PPArgs &a, int need, hipStream_t st, std::integer_sequence<int, TWS...>)
{
    hipError_t e = hipErrorInvalidValue;
    bool done = false;
    auto one = [&](auto twc) {
        constexpr int TW = decltype(twc)::value;
        if constexpr (TW <= PP_TW<KP>) {
            if (!done && need <= TW) {
                hipLaunchKernelGGL((pp_gram_kernel<KP, TW>), dim3(nblk(a.rows, 16), a.splits), dim3(256), 0, st, a);
                e = hipGetLastError();
                done = true;
            }
        }
    };
    (one(std::integral_constant<int, TWS>{}), ...);
    return e;
}

template <int KP>
static hipError_t pp_gram(const PPArgs &a, hipStream_t st)
{
    const int nt = (a.k + 3) / 4, need = (nt * (nt + 1) / 2 + 3) / 4;
    hipError_t e = pp_gram_launch<KP>(a, need, st, std::integer_sequence<int, 1, 2, 3, 4, 6, 9, 12, 17, 23, 34>{});
    if (e != hipSuccess) return e;
    if (a.splits > 1) {
        const int64_t len = a.rows * (int64_t)PP_GSZ<KP>, stride = (a.rows + 15) / 16 * 16 * (int64_t)PP_GSZ<KP>;
        hipLaunchKernelGGL(pp_reduce_kernel, dim3(nblk(len)), dim3(256), 0, st, a.gpart, a.splits, len, stride,
                           a.gram);
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
    // 64 / KP rows per wavefront, KP lanes each: the rows share every barrier
    // of the factorization and the solves
    constexpr int NR = 64 / KP;
    // Per row, the lower triangle of the first k coordinates, packed by rows
    // (entry (r, c), c <= r < k, at r (r + 1) / 2 + c), then the right-hand
    // side (KP): pp_solve_lds_doubles(k) doubles, sized at launch, so the LDS
    // follows the rank and the wavefronts per CU grow as it falls.
    extern __shared__ double pp_solve_lds[];
    const int sub = threadIdx.x / KP, lane = threadIdx.x % KP;
    const int k = a.k, tri = k * (k + 1) / 2;
    double *sM = pp_solve_lds + (size_t)sub * (tri + KP);
    double *sR = sM + tri;
    auto at = [](int r, int c) { return r * (r + 1) / 2 + c; };
    const int64_t irow = (int64_t)blockIdx.x * NR + sub;
    const int64_t i = min<int64_t>(irow, a.rows - 1);   // a row past the end repeats the last, not stored
    const float *g = a.gram + i * GSZ;
    const double al = (double)a.alpha[i];
    const double h = 1.0 / (2.0 * al);
    // the lower triangle from the upper tiles that meet the rank (G is
    // symmetric: tile entry (rr, cc) is entry (cc, rr)); tile coordinates
    // past k are padding
    const int nt = pp_nt(k), ut = nt * (nt + 1) / 2;
    for (int e = lane; e < ut * 16; e += KP) {
        int ta, tb;
        tile_of_rt(e >> 4, nt, ta, tb);
        const int rr = 4 * ta + ((e >> 2) & 3), cc = 4 * tb + (e & 3);
        if (rr < k && cc < k) sM[at(max(rr, cc), min(rr, cc))] = (double)g[e];
    }
    __syncthreads();
    if (lane < k) sM[at(lane, lane)] += h;
    __syncthreads();
    // Cholesky, lower triangle in place.  Coordinates past k take no part:
    // their right-hand side and solution are 0.
    for (int j = 0; j < k; ++j) {
        if (lane == j) {
            double d = sM[at(j, j)];
            for (int l = 0; l < j; ++l) d -= sM[at(j, l)] * sM[at(j, l)];
            sM[at(j, j)] = sqrt(d);
        }
        __syncthreads();
        if (lane > j && lane < k) {
            double s = sM[at(lane, j)];
            for (int l = 0; l < j; ++l) s -= sM[at(lane, l)] * sM[at(j, l)];
            sM[at(lane, j)] = s / sM[at(j, j)];
        }
        __syncthreads();
    }
    const double bc = lane < k ? (double)g[PP_BOFF<KP> + lane] : 0.0;
    double x = lane < k ? (double)a.U[i * k + lane] : 0.0;
    for (int it = 0; it < a.inner; ++it) {
        sR[lane] = bc + h * x;
        __syncthreads();
        for (int j = 0; j < k; ++j) {         // L y = rhs
            if (lane == j) sR[j] = sR[j] / sM[at(j, j)];
            __syncthreads();
            if (lane > j && lane < k) sR[lane] -= sM[at(lane, j)] * sR[j];
            __syncthreads();
        }
        for (int j = k - 1; j >= 0; --j) {    // L^T x = y
            if (lane == j) sR[j] = sR[j] / sM[at(j, j)];
            __syncthreads();
            if (lane < j) sR[lane] -= sM[at(j, lane)] * sR[j];
            __syncthreads();
        }
        x = lane < k ? prox_elem64(a.reg, al, sR[lane], lane) : 0.0;
        __syncthreads();
    }
    if (lane < k && irow < a.rows) a.trial[i * k + lane] = (float)x;
}

// LDS of one solve workgroup: 64 / kp rows, each the packed lower triangle of
// k coordinates and a right-hand side of kp.
static size_t pp_solve_lds_bytes(int k, int kp)
{
    return sizeof(double) * (size_t)(64 / kp) * ((size_t)k * (k + 1) / 2 + kp);
}

hipError_t launch_pp_solve(const PPArgs &a, hipStream_t st)
{
    if (a.k < 1 || a.k > a.kp) return hipErrorInvalidValue;
    if (a.rows <= 0) return hipSuccess;
    switch (a.kp) {
    case 16: hipLaunchKernelGGL(pp_solve_kernel<16>, dim3((unsigned)((a.rows + 3) / 4)), dim3(64), pp_solve_lds_bytes(a.k, 16), st, a); break;
    case 32: hipLaunchKernelGGL(pp_solve_kernel<32>, dim3((unsigned)((a.rows + 1) / 2)), dim3(64), pp_solve_lds_bytes(a.k, 32), st, a); break;
    case 64: hipLaunchKernelGGL(pp_solve_kernel<64>, dim3((unsigned)a.rows), dim3(64), pp_solve_lds_bytes(a.k, 64), st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- check pass: old and trial loss sums per row (split partials), then the rule
// On the matrix cores: per 16-row panel and 16-column tile, Z = U . V^T and
// Z+ = U+ . V^T (fp32 16x16x4 products over the rank), then w (a - z)^2 per
// observed entry.  Columns go in chunks of 64 staged in LDS, one 16-column
// tile per wavefront; each lane sums its rows over its columns, and the sums
// over the sixteen columns of a tile and over the four wavefronts are taken
// in a fixed order at the end.
template <int KP>
__global__ __launch_bounds__(256) void pp_check_kernel(PPArgs a)
{
    constexpr int CH = 64, KS = KP / 4;
    __shared__ float sV[CH][KP + 4];
    __shared__ float sT[16][CH + 4];
    __shared__ float sW[CH];
    __shared__ float sSum[4][16][2];
    // w as a scalar: the tile tests below are then scalar branches, not exec-mask ones
    const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int li = lane & 15, g = lane >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * 16;
    const int64_t per = (a.cols + a.splits - 1) / a.splits;
    const int64_t c0 = (int64_t)blockIdx.y * per, c1 = min<int64_t>(a.cols, c0 + per);
    const int k = a.k;
    // A operands: row li of the panel, coordinates 4 kk + g (old and trial rows)
    float uo[KS], ut[KS];
    {
        const int64_t i = i0 + li;
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const int c = 4 * kk + g;
            const bool ok = i < a.rows && c < k;
            uo[kk] = ok ? a.U[i * k + c] : 0.0f;
            ut[kk] = ok ? a.trial[i * k + c] : 0.0f;
        }
    }
    // this lane's rows 4 g + r: their weights and sums
    float wr[4], lo[4] = {0.f, 0.f, 0.f, 0.f}, lt[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + 4 * g + r;
        wr[r] = (a.wrow && i < a.rows) ? a.wrow[i] : 1.0f;
    }
    PPChunk<KP> chunk;
    if (c0 < c1) chunk.load(a, i0, c0, c1);
    for (int64_t j0 = c0; j0 < c1; j0 += CH) {
        __syncthreads();
        chunk.store(sV, sT, sW);
        __syncthreads();
        if (j0 + CH < c1) chunk.load(a, i0, j0 + CH, c1);   // in flight while this chunk computes
        // this wavefront's tile of the chunk: columns 16 w .. 16 w + 15
        const int jc = 16 * w + li;               // B operand column, and this lane's column of Z
        f32x4 zo = {0.f, 0.f, 0.f, 0.f}, zt = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const float bv = sV[jc][4 * kk + g];
            zo = __builtin_amdgcn_mfma_f32_16x16x4f32(uo[kk], bv, zo, 0, 0, 0);
            zt = __builtin_amdgcn_mfma_f32_16x16x4f32(ut[kk], bv, zt, 0, 0, 0);
        }
        const float wc = sW[jc];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float av = sT[4 * g + r][jc];      // unobserved, or past the rows / columns: NaN
            const float d = av - zo[r], dt = av - zt[r];
            const float ww = wr[r] * wc;
            lo[r] += av == av ? ww * d * d : 0.0f;
            lt[r] += av == av ? ww * dt * dt : 0.0f;
        }
    }
    // rows 4 g + r: the sixteen columns of the lane's group, then the wavefronts
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        lo[r] = row16_sum(lo[r]);
        lt[r] = row16_sum(lt[r]);
    }
    if (li == 0)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            sSum[w][4 * g + r][0] = lo[r];
            sSum[w][4 * g + r][1] = lt[r];
        }
    __syncthreads();
    if (t < 16) {
        const int64_t i = i0 + t;
        if (i < a.rows) {
            float so = 0.0f, st = 0.0f;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                so += sSum[v][t][0];
                st += sSum[v][t][1];
            }
            float *fp = a.fpart + ((int64_t)blockIdx.y * a.rows + i) * 2;
            fp[0] = so;
            fp[1] = st;
        }
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
    case 16: hipLaunchKernelGGL(pp_check_kernel<16>, dim3(nblk(a.rows, 16), a.splits), dim3(256), 0, st, a); break;
    case 32: hipLaunchKernelGGL(pp_check_kernel<32>, dim3(nblk(a.rows, 16), a.splits), dim3(256), 0, st, a); break;
    case 64: hipLaunchKernelGGL(pp_check_kernel<64>, dim3(nblk(a.rows, 16), a.splits), dim3(256), 0, st, a); break;
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
// Two launches in a fixed order: PP_FIN_BLOCKS workgroups each sum a
// contiguous range of the rows' and the columns' values into part (F, row
// rejections, column rejections per workgroup), then one workgroup sums the
// parts in order.
constexpr int PP_FIN_BLOCKS = 128;

__global__ __launch_bounds__(256) void pp_finalize_part_kernel(const double *rx, const int32_t *jx, int64_t m,
                                                               const double *ry, const int32_t *jy, int64_t n,
                                                               double *part)
{
    __shared__ double sF[256];
    __shared__ double sa[256], sb[256];
    const int64_t mb = (m + PP_FIN_BLOCKS - 1) / PP_FIN_BLOCKS, nb = (n + PP_FIN_BLOCKS - 1) / PP_FIN_BLOCKS;
    const int64_t m0 = blockIdx.x * mb, m1 = min<int64_t>(m, m0 + mb);
    const int64_t n0 = blockIdx.x * nb, n1 = min<int64_t>(n, n0 + nb);
    double F = 0.0, ra = 0.0, rb = 0.0;
    for (int64_t q = n0 + threadIdx.x; q < n1; q += 256) { F += ry[q]; rb += jy[q]; }
    for (int64_t q = m0 + threadIdx.x; q < m1; q += 256) { F += rx[q]; ra += jx[q]; }
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
        part[blockIdx.x] = sF[0];
        part[PP_FIN_BLOCKS + blockIdx.x] = sa[0];   // counts below 2^53: exact in double
        part[2 * PP_FIN_BLOCKS + blockIdx.x] = sb[0];
    }
}

__global__ __launch_bounds__(PP_FIN_BLOCKS) void pp_finalize_kernel(const double *part, double *stats,
                                                                    long long *istats, double *history, int32_t sweep)
{
    __shared__ double sF[PP_FIN_BLOCKS], sa[PP_FIN_BLOCKS], sb[PP_FIN_BLOCKS];
    sF[threadIdx.x] = part[threadIdx.x];
    sa[threadIdx.x] = part[PP_FIN_BLOCKS + threadIdx.x];
    sb[threadIdx.x] = part[2 * PP_FIN_BLOCKS + threadIdx.x];
    __syncthreads();
    for (int o = PP_FIN_BLOCKS / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sF[threadIdx.x] += sF[threadIdx.x + o];
            sa[threadIdx.x] += sa[threadIdx.x + o];
            sb[threadIdx.x] += sb[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        stats[0] = sF[0];
        istats[0] = (long long)sa[0];
        istats[1] = (long long)sb[0];
        if (history) history[sweep] = sF[0];
    }
}

int pp_finalize_part_doubles() { return 3 * PP_FIN_BLOCKS; }

hipError_t launch_pp_finalize(const double *rowobj_x, const int32_t *rej_x, int64_t m, const double *rowobj_y,
                              const int32_t *rej_y, int64_t n, double *part, double *stats, long long *istats,
                              double *history, int32_t sweep, hipStream_t st)
{
    hipLaunchKernelGGL(pp_finalize_part_kernel, dim3(PP_FIN_BLOCKS), dim3(256), 0, st, rowobj_x, rej_x, m, rowobj_y,
                       rej_y, n, part);
    hipLaunchKernelGGL(pp_finalize_kernel, dim3(1), dim3(PP_FIN_BLOCKS), 0, st, part, stats, istats, history, sweep);
    return hipGetLastError();
}

}  // namespace glrm
