// Dense-layout kernels of the GLRM sweep for gfx950 (templates; instantiated
// per precision in dense_prec.hip).
//
// The table sits in the workspace as a padded copy (rows to a multiple of 16,
// columns to a multiple of 16) in which every unobserved entry is a quiet NaN,
// so one 4-byte load gives both the value and the observation bit.
//
// Work decomposition: a persistent workgroup of W wavefronts walks 16-row
// panels.  The panel's columns are cut into 16-wide tiles and tile t belongs
// to wavefront t mod W for the whole launch, so each wavefront keeps its
// tiles' Y operands and its per-column accumulators (column objective, Y
// gradient) in registers across panels.  The next panel's table tiles travel
// straight from HBM into LDS while the current one computes.
//
// Matrix-core products per 16 x 16 tile (i = row of the panel, j = column):
//   z     Z^T(16j x 16i) = Y_tile(16j x kp) . X_panel^T        -> lane holds z(i=l%16, j=4(l/16)+r)
//   S3    dX(16i x 16kc) += G(16i x 16j) . Y_tile(16j x 16kc)   (G straight from the z layout)
//   S6    Z(16i x 16j) = X_panel . Y_tile^T                     -> lane holds z(i=4(l/16)+r, j=l%16)
//         dY(16j x 16kc) += G^T(16j x 16i) . X(16i x 16kc)      (G straight from that layout)
// The k index each lane feeds is a free choice as long as both operands use
// the same one: lane group g = l/16 feeds the contiguous run k = g*kp/4 ...
// (g+1)*kp/4 - 1, which makes every operand load one contiguous vector.
#pragma once

#include "glrm_device.h"
#include "glrm_kernels.h"

namespace glrm {

constexpr int GS = 20;           // row stride (floats) of the per-wave transpose tiles

// ---------------------------------------------------------------------------
// operand fragments
// ---------------------------------------------------------------------------
template <int KP, int PREC>
struct Frag {
    // lane group g's run of kp/4 coordinates, packed: fp32 values, or bf16
    // high / low parts in vectors of eight (four at kp = 16)
    static constexpr int C = KP / 4;
    static constexpr int NV = C >= 8 ? C / 8 : 1;
    float f[PREC == P_FP32 ? C : 1];
    bf16x8 hi[PREC == P_FP32 ? 1 : NV];
    bf16x8 lo[PREC == P_BF16 ? NV : 1];
};

// From fp32 values (LDS panel row or registers).
template <int KP, int PREC>
__device__ __forceinline__ void frag_from_f32(Frag<KP, PREC> &fr, const float *src)
{
#pragma unroll
    for (int q = 0; q < KP / 4; ++q) {
        const float v = src[q];
        if constexpr (PREC == P_FP32) {
            fr.f[q] = v;
        } else if constexpr (PREC == P_BF16) {
            __bf16 h, l;
            split_bf16(v, h, l);
            fr.hi[q / 8][q % 8] = h;
            fr.lo[q / 8][q % 8] = l;
        } else {
            fr.hi[q / 8][q % 8] = to_bf16(v);
        }
    }
}

// Row j of a padded shadow of Y (or Y+) in global memory, lane group g's run.
template <int KP, int PREC>
__device__ __forceinline__ void frag_load_y(Frag<KP, PREC> &fr, const YShadow &ys, int64_t j, int g)
{
    constexpr int C = KP / 4;
    if constexpr (PREC == P_FP32) {
        const float4 *p = reinterpret_cast<const float4 *>(ys.f32 + j * KP + g * C);
#pragma unroll
        for (int q = 0; q < C / 4; ++q) {
            float4 v = p[q];
            fr.f[4 * q + 0] = v.x; fr.f[4 * q + 1] = v.y; fr.f[4 * q + 2] = v.z; fr.f[4 * q + 3] = v.w;
        }
    } else {
        const __bf16 *ph = ys.hi + j * KP + g * C;
        const __bf16 *pl = ys.lo + j * KP + g * C;
        if constexpr (C == 4) {
            uint2 h = *reinterpret_cast<const uint2 *>(ph);
            uint4 hv = {h.x, h.y, 0u, 0u};
            fr.hi[0] = __builtin_bit_cast(bf16x8, hv);
            if constexpr (PREC == P_BF16) {
                uint2 l = *reinterpret_cast<const uint2 *>(pl);
                uint4 lv = {l.x, l.y, 0u, 0u};
                fr.lo[0] = __builtin_bit_cast(bf16x8, lv);
            }
        } else {
#pragma unroll
            for (int q = 0; q < C / 8; ++q) {
                fr.hi[q] = __builtin_bit_cast(bf16x8, reinterpret_cast<const uint4 *>(ph)[q]);
                if constexpr (PREC == P_BF16)
                    fr.lo[q] = __builtin_bit_cast(bf16x8, reinterpret_cast<const uint4 *>(pl)[q]);
            }
        }
    }
}

// Z^T tile = Y_tile . X_panel^T.  Split bf16: the two small cross terms first.
template <int KP>
__device__ __forceinline__ f32x4 mfma_vec(const bf16x8 *a, const bf16x8 *b, f32x4 acc)
{
    if constexpr (KP == 16) {
        const uint4 av = __builtin_bit_cast(uint4, a[0]), bv = __builtin_bit_cast(uint4, b[0]);
        const uint2 a2 = {av.x, av.y}, b2 = {bv.x, bv.y};
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(i16x4, a2), __builtin_bit_cast(i16x4, b2),
                                                         acc, 0, 0, 0);
    } else {
#pragma unroll
        for (int q = 0; q < KP / 32; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[q], b[q], acc, 0, 0, 0);
        return acc;
    }
}

template <int KP, int PREC>
__device__ __forceinline__ f32x4 zprod(const Frag<KP, PREC> &y, const Frag<KP, PREC> &x)
{
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    if constexpr (PREC == P_FP32) {
#pragma unroll
        for (int q = 0; q < KP / 4; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(y.f[q], x.f[q], acc, 0, 0, 0);
    } else {
        if constexpr (PREC == P_BF16) {
            acc = mfma_vec<KP>(y.lo, x.hi, acc);
            acc = mfma_vec<KP>(y.hi, x.lo, acc);
        }
        acc = mfma_vec<KP>(y.hi, x.hi, acc);
    }
    return acc;
}

// Transpose the wave's 16x16 G tile in registers: lane li + 16 g holds
// G[li][4g + r] in G[r] and receives G[4g + r][li] in gT[r].  First a 4x4
// transpose inside every quad of lanes (the quad's four rows of one 4x4 block,
// across the four registers) with DPP quad permutations; then lane
// jj + 4 bj + 16 bi takes the registers of lane jj + 4 bi + 16 bj (one
// ds_bpermute per register).  No LDS memory is touched, so nothing here waits
// for the next panel's direct-to-LDS loads.
__device__ __forceinline__ void transpose_g(const float (&G)[4], float (&gT)[4])
{
    const int lane = threadIdx.x & 63;
    float m[4] = {G[0], G[1], G[2], G[3]};
    {   // quad lanes q and q ^ 2 exchange registers r + 2 / r
        const bool hi = (lane & 2) != 0;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const float a = m[r], c = m[r + 2];
            const float pa = dpp_mov<0x4E>(a), pc = dpp_mov<0x4E>(c);   // quad_perm [2,3,0,1]
            m[r] = hi ? pc : a;
            m[r + 2] = hi ? c : pa;
        }
    }
    {   // quad lanes q and q ^ 1 exchange registers r + 1 / r
        const bool hi = (lane & 1) != 0;
#pragma unroll
        for (int r = 0; r < 4; r += 2) {
            const float a = m[r], c = m[r + 1];
            const float pa = dpp_mov<0xB1>(a), pc = dpp_mov<0xB1>(c);   // quad_perm [1,0,3,2]
            m[r] = hi ? pc : a;
            m[r + 1] = hi ? c : pa;
        }
    }
    const int src = (lane & 3) | (((lane >> 4) & 3) << 2) | (((lane >> 2) & 3) << 4);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        gT[r] = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(4 * src, __builtin_bit_cast(int, m[r])));
}

// Wavefronts per workgroup of the two passes over the table (xstep_waves,
// ycheck_waves).  A wavefront's tiles' Y operands stay resident for the whole
// launch and its column accumulators live in registers.
template <int KP>
constexpr int NWX_OF = xstep_waves(KP);
template <int KP>
constexpr int NTX_OF = 64 * NWX_OF<KP>;
template <int KP>
constexpr int NWY_OF = ycheck_waves(KP);
template <int KP>
constexpr int NWG_OF = grad_waves(KP);
template <int KP>
constexpr int NTG_OF = 64 * NWG_OF<KP>;
template <int KP>
constexpr int NTY_OF = 64 * NWY_OF<KP>;

// ---------------------------------------------------------------------------
// panel staging: the next 16-row panel's table tiles, X rows and step sizes
// travel straight from HBM into an LDS buffer while the current panel
// computes (global_load_lds: lane l's 16 or 4 bytes land at base + l * size).
// A panel reads only the buffer it computes on.  After a direct-to-LDS load
// the compiler waits for it before any LDS access it cannot prove unrelated,
// so the passes either read their tiles before issuing the prefetch
// (trial-column pass) or hand the buffers over as restrict pointers (row
// pass).
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

__device__ __forceinline__ void lds_dma16(const void *src, void *wave_dst)
{
    __builtin_amdgcn_global_load_lds((glb_void_t *)src, (lds_void_t *)wave_dst, 16, 0, 0);
}

__device__ __forceinline__ void lds_dma4(const void *src, void *wave_dst)
{
    __builtin_amdgcn_global_load_lds((glb_void_t *)src, (lds_void_t *)wave_dst, 4, 0, 0);
}

template <int KP, int TPW, int NW>
struct PanelBuf {
    float4 apan[NW][TPW * 64];   // wavefront w's tiles: [tile slot][lane]
    float xrow[16 * KP];         // the panel's X rows, contiguous (16 * k floats)
    float alpha[16];
};

// Where a tile's entries sit in its 1 KB slot.  Lane l = li + 16g reads row
// li's columns 4g .. 4g+3 as one 16-byte word (the plain read), and in S6 the
// rows 4g .. 4g+3 of column li (the transposed read).  Row i's columns
// 4q .. 4q+3 are staged in word 16q + ((i + q) & 15): each quarter-wave's plain
// reads then fall on 16 distinct words, and each 4-byte step of the transposed
// read on 64 distinct banks (stored in order, row i's words sat in one bank
// group per q, a 4-way conflict).
__device__ __forceinline__ int tile_word(int row, int q) { return 16 * q + ((row + q) & 15); }

// The staged word of lane l's plain read.  Only the row pass reads its tiles
// transposed, so only it stages them in this order (SWZ); the other passes
// keep row i's block q in word i + 16q, which they read in lane order.
template <bool SWZ>
__device__ __forceinline__ int tile_slot(int lane) { return SWZ ? tile_word(lane & 15, lane >> 4) : lane; }

// Loads of panel p into `pb`: tile slot s of this wavefront (lane l fills
// word l, with the row whose block g belongs there) ...
template <int KP, int TPW, int NW, bool SWZ = false>
__device__ __forceinline__ void stage_tile(PanelBuf<KP, TPW, NW> &pb, const float *Ap, int64_t ldp, int nt, int64_t p,
                                           int w, int lane, int s, int tile0 = 0)
{
    const int li = lane & 15, g = lane >> 4;
    const int row = SWZ ? (li - g) & 15 : li;   // tile_word(row, g) == lane under SWZ
    const int t = min(tile0 + w + NW * s, nt - 1);
    lds_dma16(Ap + (p * 16 + row) * ldp + 4 * g + 16 * t, &pb.apan[w][s * 64]);
}

// ... and the X rows and step sizes (spread over the wavefronts).
template <int KP, int TPW, int NW>
__device__ __forceinline__ void stage_rows(PanelBuf<KP, TPW, NW> &pb, const float *X, int64_t m, int k,
                                           const float *alpha, int64_t p, int w, int lane)
{
    const int64_t i0 = p * 16;
    const int64_t rows = min<int64_t>(16, m - i0);
    const int nx = (int)(rows * k);            // valid floats of the row block
    const float *xb = X + i0 * k;
    for (int q = w; q * 64 < nx; q += NW)
        if (q * 64 + lane < nx) lds_dma4(xb + q * 64 + lane, &pb.xrow[q * 64]);
    if (alpha && w == NW - 1 && lane < rows) lds_dma4(alpha + i0 + lane, &pb.alpha[0]);
}

// All loads of panel p into `pb` (every wavefront issues its own tiles).
template <int KP, int TPW, int NW, bool SWZ = false>
__device__ __forceinline__ void stage_panel(PanelBuf<KP, TPW, NW> &pb, const float *Ap, int64_t ldp, int nt,
                                            const float *X, int64_t m, int k, const float *alpha, int64_t p,
                                            int w, int lane, int tile0 = 0)
{
#pragma unroll
    for (int s = 0; s < TPW; ++s) stage_tile<KP, TPW, NW, SWZ>(pb, Ap, ldp, nt, p, w, lane, s, tile0);
    stage_rows<KP, TPW, NW>(pb, X, m, k, alpha, p, w, lane);
}

// The lane's four table entries of tile slot s.  A slot past the last tile
// (its wavefront has fewer tiles than slots) reads as unobserved, so every
// slot runs the same code and contributes exactly zero.
__device__ __forceinline__ float4 tile_entries(const float4 *apan, int s, int lane, bool valid)
{
    const float4 v = apan[s * 64 + lane];
    const float qnan = __builtin_nanf("");
    return valid ? v : float4{qnan, qnan, qnan, qnan};
}

// The lane's four table entries in the layout of X . Y^T products: rows
// 4g + r of column li of tile slot s (row 4g + r's block li >> 2, entry li & 3),
// in the row pass's staging order.
__device__ __forceinline__ float4 tile_entries_t(const float4 *apan, int s, int li, int g)
{
    const int q = li >> 2;
    const float *b = reinterpret_cast<const float *>(apan) + s * 256 + (li & 3);
    return float4{b[4 * tile_word(4 * g + 0, q)], b[4 * tile_word(4 * g + 1, q)], b[4 * tile_word(4 * g + 2, q)],
                  b[4 * tile_word(4 * g + 3, q)]};
}

__device__ __forceinline__ void wait_staged()
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Resident operands of the wavefront's tiles (Y is fixed during a half-step).
template <int KP, int PREC>
struct YtFrag {
    float4 f[PREC == P_FP32 ? KP / 16 : 1];
    i16x4 b[PREC == P_FP32 ? 1 : KP / 16];
};

template <int KP, int PREC>
__device__ __forceinline__ void ytfrag_load(YtFrag<KP, PREC> &yt, const YShadow &ys, int64_t ldp, int64_t j0, int li,
                                            int g)
{
#pragma unroll
    for (int kb = 0; kb < KP / 16; ++kb) {
        const int64_t off = (int64_t)(16 * kb + li) * ldp + j0 + 4 * g;
        if constexpr (PREC == P_FP32) yt.f[kb] = *reinterpret_cast<const float4 *>(ys.t32 + off);
        else *reinterpret_cast<uint2 *>(&yt.b[kb]) = *reinterpret_cast<const uint2 *>(ys.tb + off);
    }
}

// S3 with a resident operand: dX(16i x 16kc) += G(16i x 16j) . Y_tile(16j x 16kc).
template <int KP, int PREC>
__device__ __forceinline__ void s3_resident(f32x4 (&dx)[KP / 16], const float (&G)[4], const YtFrag<KP, PREC> &yt)
{
    if constexpr (PREC == P_FP32) {
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb) {
            dx[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(G[0], yt.f[kb].x, dx[kb], 0, 0, 0);
            dx[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(G[1], yt.f[kb].y, dx[kb], 0, 0, 0);
            dx[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(G[2], yt.f[kb].z, dx[kb], 0, 0, 0);
            dx[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(G[3], yt.f[kb].w, dx[kb], 0, 0, 0);
        }
    } else {
        const i16x4 av = pack_bf16x4(G[0], G[1], G[2], G[3]);
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb)
            dx[kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, yt.b[kb], dx[kb], 0, 0, 0);
    }
}

// The S6 operand X(16i x 16kc) of a panel, from the transposed accepted rows
// (xat, [kc][i]): fixed for the whole panel, so it is read and rounded once.
template <int KP, int PREC>
struct XatFrag {
    float4 f[PREC == P_FP32 ? KP / 16 : 1];
    i16x4 b[PREC == P_FP32 ? 1 : KP / 16];
};

template <int KP, int PREC>
__device__ __forceinline__ void xatfrag_load(XatFrag<KP, PREC> &xa, const float *xat, int li, int g)
{
#pragma unroll
    for (int kb = 0; kb < KP / 16; ++kb) {
        const float4 b = *reinterpret_cast<const float4 *>(xat + (16 * kb + li) * GS + 4 * g);
        if constexpr (PREC == P_FP32) xa.f[kb] = b;
        else xa.b[kb] = pack_bf16x4(b.x, b.y, b.z, b.w);
    }
}

// S6 with the panel operand in registers: dY(16j x 16kc) += G^T(16j x 16i) . X(16i x 16kc).
template <int KP, int PREC>
__device__ __forceinline__ void s6_resident(f32x4 (&dy)[KP / 16], const float (&gT)[4], const XatFrag<KP, PREC> &xa)
{
    if constexpr (PREC == P_FP32) {
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb) {
            dy[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(gT[0], xa.f[kb].x, dy[kb], 0, 0, 0);
            dy[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(gT[1], xa.f[kb].y, dy[kb], 0, 0, 0);
            dy[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(gT[2], xa.f[kb].z, dy[kb], 0, 0, 0);
            dy[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(gT[3], xa.f[kb].w, dy[kb], 0, 0, 0);
        }
    } else {
        const i16x4 av = pack_bf16x4(gT[0], gT[1], gT[2], gT[3]);
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb)
            dy[kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, xa.b[kb], dy[kb], 0, 0, 0);
    }
}

// HALF (quadratic loss only): g is half the derivative, z - a; the caller
// doubles its reductions instead (exact: a power of two).
template <int K, bool WANT_G, bool HALF = false>
__device__ __forceinline__ void tile4(int lev, float par, const f32x4 &z, const float (&a4)[4], float (&l)[4],
                                      float (&g)[4])
{
    if constexpr (K == L_QUAD && WANT_G && HALF) {
        // an unobserved entry (NaN) gives d = 0, hence l = g = 0
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float d = a4[r] == a4[r] ? z[r] - a4[r] : 0.0f;
            l[r] = d * d;
            g[r] = d;
        }
        return;
    }
    if constexpr (K == L_QUAD && !WANT_G) {
        // only an unobserved entry (NaN in the table) is masked; a NaN
        // product keeps a NaN loss, so such a trial point is never accepted
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float d = z[r] - a4[r];
            l[r] = a4[r] == a4[r] ? d * d : 0.0f;
            g[r] = 0.0f;
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float lr = 0.f, gr = 0.f;
        if (a4[r] == a4[r]) {
            if constexpr (WANT_G) loss_lg_k<K>(lev, par, z[r], a4[r], lr, gr);
            else lr = loss_l_k<K>(lev, par, z[r], a4[r]);
        }
        l[r] = lr;
        g[r] = gr;
    }
}

// Losses (and derivatives) of four entries under a per-column loss table.
// tc >= 0: the tile's sixteen columns share loss tc.  tc < 0: codes per entry
// (cd).  Inlined into every tile, phase and panel buffer, the five loss kinds
// make a pass with 8 or 16 tiles per wavefront 0.2-0.8 MB of code, far beyond
// the instruction cache; those passes call one shared copy instead
// (tile_loss_table_call), the smaller ones inline it, which measured faster.
struct LG4 {
    f32x4 l, g;
};

template <bool WANT_G>
__device__ __forceinline__ LG4 tile_loss_table(const LossTab *tab, int tc, int4 cd, f32x4 z, float4 av)
{
    const float a4[4] = {av.x, av.y, av.z, av.w};
    float l[4], g[4];
    if (tc >= 0) {
        const int kind = __builtin_amdgcn_readfirstlane(tab->kind[tc]);
        const int lev = __builtin_amdgcn_readfirstlane(tab->levels[tc]);
        const float par = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, tab->param[tc])));
        switch (kind) {
        case L_QUAD: tile4<L_QUAD, WANT_G>(lev, par, z, a4, l, g); break;
        case L_HUBER: tile4<L_HUBER, WANT_G>(lev, par, z, a4, l, g); break;
        case L_LOGISTIC: tile4<L_LOGISTIC, WANT_G>(lev, par, z, a4, l, g); break;
        case L_HINGE: tile4<L_HINGE, WANT_G>(lev, par, z, a4, l, g); break;
        default: tile4<L_ORDINAL, WANT_G>(lev, par, z, a4, l, g); break;
        }
    } else {
        const int c4[4] = {cd.x, cd.y, cd.z, cd.w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float lr = 0.f, gr = 0.f;
            if (a4[r] == a4[r]) {
                const int q = c4[r];
                if constexpr (WANT_G) loss_lg(tab->kind[q], tab->levels[q], tab->param[q], z[r], a4[r], lr, gr);
                else lr = loss_l(tab->kind[q], tab->levels[q], tab->param[q], z[r], a4[r]);
            }
            l[r] = lr;
            g[r] = gr;
        }
    }
    return LG4{f32x4{l[0], l[1], l[2], l[3]}, f32x4{g[0], g[1], g[2], g[3]}};
}

// Scale of the derivatives tile_loss<LK> returns (see tile4's HALF).
template <int LK>
constexpr float GRAD_SCALE = LK == L_QUAD ? 2.0f : 1.0f;

template <bool WANT_G>
__device__ __attribute__((noinline)) LG4 tile_loss_table_call(const LossTab *tab, int tc, int4 cd, f32x4 z,
                                                              float4 av)
{
    return tile_loss_table<WANT_G>(tab, tc, cd, z, av);
}

// Losses (and, with WANT_G, derivatives) of the lane's four entries of tile t.
// LK >= 0: every column has loss kind LK (compile time).  LK < 0: the table
// (tile_loss_table).  TRANS: the four entries are rows 4g + r of column
// 16t + li (the layout of X . Y^T products) instead of row li, columns
// 16t + 4g + r.
//
// Under a per-column loss table each entry's loss and derivative are scaled
// by its column's weight (all 1 unless the caller gave weights), staged in LDS
// beside the loss codes (s_colw, indexed like s_codes): a global load here
// would make the wait for its data also wait for the next panel's
// direct-to-LDS loads, issued before it, and take the prefetch out of the
// tile loop.
template <int LK, bool WANT_G, bool TRANS = false, int TPW = 1>
__device__ __forceinline__ void tile_loss(const LossU &lu, const LossTab &tab, const uint8_t *s_codes,
                                          const int8_t *s_tcode, int t, const f32x4 &z, const float4 &av,
                                          float (&l)[4], float (&g)[4], const float *s_colw)
{
    if constexpr (LK >= 0) {
        const float a4[4] = {av.x, av.y, av.z, av.w};
        tile4<LK, WANT_G, LK == L_QUAD>(lu.levels, lu.param, z, a4, l, g);
    } else {
        const int tc = __builtin_amdgcn_readfirstlane((int)s_tcode[t]);
        int4 cd = {0, 0, 0, 0};
        if (tc < 0) {
            const int lane = threadIdx.x & 63;
            if constexpr (TRANS) {
                const int c = s_codes[16 * t + (lane & 15)];
                cd = int4{c, c, c, c};
            } else {
                const uchar4 c = *reinterpret_cast<const uchar4 *>(s_codes + 16 * t + 4 * (lane >> 4));
                cd = int4{c.x, c.y, c.z, c.w};
            }
        }
        LG4 r;
        if constexpr (TPW <= 4) r = tile_loss_table<WANT_G>(&tab, tc, cd, z, av);
        else r = tile_loss_table_call<WANT_G>(&tab, tc, cd, z, av);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            l[q] = r.l[q];
            g[q] = r.g[q];
        }
        // unconditional (the weights are all 1 without a caller's weights): a
        // branch here would sit between a matrix-core product and its read
        const int lane = threadIdx.x & 63;
        float w[4];
        if constexpr (TRANS) {
            const float wc = s_colw[16 * t + (lane & 15)];
            w[0] = w[1] = w[2] = w[3] = wc;
        } else {
            const float4 w4 = *reinterpret_cast<const float4 *>(s_colw + 16 * t + 4 * (lane >> 4));
            w[0] = w4.x; w[1] = w4.y; w[2] = w4.z; w[3] = w4.w;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            l[q] *= w[q];
            g[q] *= w[q];
        }
    }
}

// The per-column weights of a loss table's columns c0 .. c0 + count - 1
// (clamped to the padded width, as the codes), into LDS.
__device__ __forceinline__ void stage_colw(const LossTab &lt, int64_t c0, int count, int64_t ldp, float *s_colw,
                                           int nthreads)
{
    for (int j = threadIdx.x; j < count; j += nthreads)
        s_colw[j] = lt.colw ? lt.colw[min<int64_t>(c0 + j, ldp - 1)] : 1.0f;
}

// Per-tile loss codes: the tile's code when its sixteen columns share one
// loss, else -1.
__device__ __forceinline__ void tile_codes(const uint8_t *s_codes, int nt, int8_t *s_tcode, int nthreads)
{
    for (int t = threadIdx.x; t < nt; t += nthreads) {
        const uint8_t c0 = s_codes[16 * t];
        bool same = true;
        for (int q = 1; q < 16; ++q) same = same && s_codes[16 * t + q] == c0;
        s_tcode[t] = same ? (int8_t)c0 : (int8_t)-1;
    }
}

// ---------------------------------------------------------------------------
// pass 1: fused X half-step (S1-S5) + Y-gradient and column-objective partials (S6)
// ---------------------------------------------------------------------------
// Row stride (floats) of the per-panel [16][kp] arrays: with kp + 4 the four
// lane groups of a fragment read, and of the S3 partial writes, fall in
// different LDS banks.
template <int KP>
constexpr int RS = KP + 4;

// Row stride of the row-gradient partials ([coordinate][row], 16 rows padded
// to 20 floats: 16-byte aligned, and the S4 reads of 16 coordinates x 4 rows
// land in distinct banks).
constexpr int RG = 20;

// Row stride of the row-objective partials (4 per wavefront, padded so the
// 64 lanes of a wavefront write to distinct banks).
template <int KP>
constexpr int RF = 4 * NWX_OF<KP> + 4;

// Where the row pass issues the next panel's loads: the X rows and step sizes
// at the start of S4, the tiles one per step of the trial-row loop (S5), so
// the fetch overlaps S5, the decisions and S6.  Its barriers inside a panel
// therefore wait on LDS only (lds_barrier).  The two panel buffers are LDS
// objects of their own, handed to the panel as restrict pointers: the
// compiler then knows the loads into one buffer cannot alias the panel's other
// LDS traffic, and issues no wait for them before those reads.  (The FP32 form
// once issued all its loads at the start of S6 instead; once S6's transposed
// reads no longer waited for the prefetch, this placement measured 5 % faster
// for it too.)
template <int KP, int TPW, int PREC>
struct XStepShared {
    float xs[16][RS<KP>];    // the accepted rows (S6 operand)
    float xp[16][RS<KP>];    // trial rows
    // row-gradient partials (S3 -> S4), [wavefront][coordinate][row]: a lane's
    // four rows of one coordinate are one 16-byte write
    alignas(16) float red_g[NWX_OF<KP>][KP][RG];
    alignas(16) float xat[KP * GS];                     // accepted X transposed ([kc][i]) for S6
    // row-objective partials at x (S2) and at the trial rows (S5): row i holds
    // wavefront w's lane group g at 4w + g, so a row reads them as float4s
    float red_f[16][RF<KP>], red_fp[16][RF<KP>];
    LossTab lt;                 // per-column loss table (mixed tables only)
    uint8_t s_codes[16 * NWX_OF<KP> * TPW];
    int8_t s_tcode[NWX_OF<KP> * TPW];
    float s_rx[16], s_rxp[16];
    float s_blk[NWX_OF<KP>];
    int s_rej[NWX_OF<KP>];
};

// S6 of one panel.  z comes from
// X . Y^T, so each lane holds rows 4g + r of column li: the loss derivatives
// are then already the transposed operand of dY += G^T . X, and the column
// objective of column li is a sum over the lane's four rows (the four lane
// groups are added once, at the end of the launch).  The LDS operands come in
// as restrict pointers so that the compiler can tell the next panel's loads,
// in flight, apart from the reads below.
template <int KP, int TPW, int PREC, int LK>
__device__ __forceinline__ void xstep_s6(const XStepArgs &a, const float4 *__restrict__ apan,
                                         const LossTab *__restrict__ lt, const uint8_t *__restrict__ s_codes,
                                         const int8_t *__restrict__ s_tcode, const float *__restrict__ s_colw,
                                         const Frag<KP, PREC> (&yfr)[TPW],
                                         const XatFrag<KP, PREC> &xa, const Frag<KP, PREC> &xaf,
                                         f32x4 (&dyacc)[TPW][KP / 16], float (&hacc)[TPW])
{
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, g = lane >> 4;
    const int nt = (int)(a.ldp / 16);
    // software pipelined: tile s + 1's entries and product are issued before
    // tile s's losses (slots past the last tile compute on stale entries and
    // are skipped), and each tile's work sits behind a uniform branch, since
    // straight-line tiles raise register pressure past what the resident
    // operands leave
    f32x4 zn = zprod<KP, PREC>(xaf, yfr[0]);
    float4 an = tile_entries_t(apan, 0, li, g);
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int t = w + NWX_OF<KP> * s;
        const f32x4 zt = zn;
        const float4 av = an;
        if (s + 1 < TPW) {
            zn = zprod<KP, PREC>(xaf, yfr[s + 1]);
            an = tile_entries_t(apan, s + 1, li, g);
        }
        if (t >= nt) continue;
        float L4[4], G[4];
        tile_loss<LK, true, true, TPW>(a.lu, *lt, s_codes, s_tcode, t, zt, av, L4, G, s_colw);
        hacc[s] += (L4[0] + L4[1]) + (L4[2] + L4[3]);
        s6_resident<KP, PREC>(dyacc[s], G, xa);
    }
}

// One 16-row panel of the fused X half-step.  Five workgroup barriers: the
// staged panel, the row-gradient partials, the trial rows, the trial
// objective partials and the accepted rows.  The next panel's loads go out
// right after the first, and the other four order LDS traffic only, so the
// prefetch streams in behind all five phases.  The row steps (S4) and the
// decisions run on the first 256 threads, sixteen lanes per row, so their row
// sums are DPP row reductions.
template <int KP, int TPW, int PREC, int LK, int BUF>
__device__ __forceinline__ void xstep_panel(const XStepArgs a, XStepShared<KP, TPW, PREC> &__restrict__ sh,
                                            PanelBuf<KP, TPW, NWX_OF<KP>> *__restrict__ pb0,
                                            PanelBuf<KP, TPW, NWX_OF<KP>> *__restrict__ pb1,
                                            const float *__restrict__ s_colw, int64_t p,
                                            int64_t p_next, const Frag<KP, PREC> (&yfr)[TPW],
                                            const YtFrag<KP, PREC> (&ytf)[TPW], f32x4 (&dyacc)[TPW][KP / 16],
                                            float (&hacc)[TPW], float &rowreg_acc, int &rej_acc)
{
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, g = lane >> 4;
    constexpr int C = KP / 4;
    const int nt = (int)(a.ldp / 16);
    const int k = a.k;
    PanelBuf<KP, TPW, NWX_OF<KP>> &cur = BUF == 0 ? *pb0 : *pb1;
    PanelBuf<KP, TPW, NWX_OF<KP>> &nxt = BUF == 0 ? *pb1 : *pb0;
    const float4 *apan = cur.apan[w];
    const int64_t i0 = p * 16;
    const int rows = (int)min<int64_t>(16, a.m - i0);
    // the row-step thread map: row ri, coordinates c0 + 16 q
    const int ri = threadIdx.x >> 4, c0 = threadIdx.x & 15;
    const bool rv = ri < rows;

    wait_staged();

    // ---- S1-S3: z, loss, derivative, row objective, row gradient ------------------
    // the panel's X rows straight from the staged block (16 x k, contiguous)
    Frag<KP, PREC> xf;
    {
        float xv[C];
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int c = g * C + q;
            xv[q] = (li < rows && c < k) ? cur.xrow[li * k + c] : 0.0f;
        }
        frag_from_f32<KP, PREC>(xf, xv);
    }
    float fpart = 0.0f;
    f32x4 dx[KP / 16];
#pragma unroll
    for (int kb = 0; kb < KP / 16; ++kb) dx[kb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // software pipelined as in S6
    f32x4 zn = zprod<KP, PREC>(yfr[0], xf);
    float4 an = apan[tile_slot<true>(lane)];
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int t = w + NWX_OF<KP> * s;
        const f32x4 z = zn;
        const float4 av = an;
        if (s + 1 < TPW) {
            zn = zprod<KP, PREC>(yfr[s + 1], xf);
            an = apan[(s + 1) * 64 + tile_slot<true>(lane)];
        }
        if (t >= nt) continue;
        float L4[4], G[4];
        tile_loss<LK, true, false, TPW>(a.lu, sh.lt, sh.s_codes, sh.s_tcode, t, z, av, L4, G, s_colw);
        fpart += (L4[0] + L4[1]) + (L4[2] + L4[3]);
        s3_resident<KP, PREC>(dx, G, ytf[s]);
    }
    sh.red_f[li][4 * w + g] = fpart;
#pragma unroll
    for (int kb = 0; kb < KP / 16; ++kb)
        *reinterpret_cast<f32x4 *>(&sh.red_g[w][16 * kb + li][4 * g]) = dx[kb];
    lds_barrier();

    // ---- S4: prox step and regularizer values ------------------------------------
    // the next panel's X rows and step sizes go out first; no matrix-core
    // product is in flight here.  Then every LDS read (unconditional: the
    // indexes stay inside the arrays), one wait, then the arithmetic.
    if (p_next >= 0) stage_rows<KP, TPW, NWX_OF<KP>>(nxt, a.X, a.m, a.k, a.alpha, p_next, w, lane);
    if (threadIdx.x < 256) {
        constexpr int Q = KP / 16;
        const float al0 = cur.alpha[ri];
        float xq[Q], gq[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int c = c0 + 16 * q;
            xq[q] = cur.xrow[ri * k + c];
            float gs = 0.0f;
#pragma unroll
            for (int v = 0; v < NWX_OF<KP>; ++v) gs += sh.red_g[v][c][ri];
            gq[q] = gs * GRAD_SCALE<LK>;
        }
        const float al = rv ? al0 : 0.0f;
        float rc = 0.0f, rcp = 0.0f;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int c = c0 + 16 * q;
            const bool ok = rv && c < k;
            const float x = ok ? xq[q] : 0.0f;
            const float xv = ok ? prox_elem(a.rx, al, x - al * gq[q], c) : 0.0f;
            sh.xp[ri][c] = xv;
            rc += ok ? reg_elem(a.rx, x, c) : 0.0f;
            rcp += ok ? reg_elem_trial(a.rx, xv, c) : 0.0f;
        }
        rc = row16_sum(rc);
        rcp = row16_sum(rcp);
        if (c0 == 0) {
            sh.s_rx[ri] = rc;
            sh.s_rxp[ri] = rcp;
        }
    }
    lds_barrier();

    // ---- S5: row objective at the trial rows ---------------------------------------
    Frag<KP, PREC> xpf;
    frag_from_f32<KP, PREC>(xpf, &sh.xp[li][g * C]);
    float fppart = 0.0f;
    // the next panel's tiles are issued one per step of this loop.  The issue is unconditional (without a next panel it reloads this
    // panel into the idle buffer): a branch between a matrix-core product and
    // the read of its result lets the taken path skip the wait states the
    // read needs.
    const int64_t p_src = p_next >= 0 ? p_next : p;
    f32x4 zn2 = zprod<KP, PREC>(yfr[0], xpf);
    float4 an2 = apan[tile_slot<true>(lane)];
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int t = w + NWX_OF<KP> * s;
        const f32x4 zp = zn2;
        const float4 av = an2;
        stage_tile<KP, TPW, NWX_OF<KP>, true>(nxt, a.Ap, a.ldp, nt, p_src, w, lane, s);
        if (s + 1 < TPW) {
            zn2 = zprod<KP, PREC>(yfr[s + 1], xpf);
            an2 = apan[(s + 1) * 64 + tile_slot<true>(lane)];
        }
        if (t >= nt) continue;
        float L4[4], G4[4];
        tile_loss<LK, false, false, TPW>(a.lu, sh.lt, sh.s_codes, sh.s_tcode, t, zp, av, L4, G4, s_colw);
        fppart += (L4[0] + L4[1]) + (L4[2] + L4[3]);
    }
    sh.red_fp[li][4 * w + g] = fppart;
    lds_barrier();

    // ---- decision per row and the accepted rows ---------------------------------------
    if (threadIdx.x < 256) {
        constexpr int Q = KP / 16;
        float4 fa[NWX_OF<KP>], fb[NWX_OF<KP>];
#pragma unroll
        for (int v = 0; v < NWX_OF<KP>; ++v) {
            fa[v] = *reinterpret_cast<const float4 *>(&sh.red_f[ri][4 * v]);
            fb[v] = *reinterpret_cast<const float4 *>(&sh.red_fp[ri][4 * v]);
        }
        const float rx = sh.s_rx[ri], rxp = sh.s_rxp[ri], al0 = cur.alpha[ri];
        float xq[Q], xpq[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            xq[q] = cur.xrow[ri * k + c0 + 16 * q];
            xpq[q] = sh.xp[ri][c0 + 16 * q];
        }
        // the same sums, in the same order, in every lane of the row
        float f = 0.0f, fp = 0.0f;
#pragma unroll
        for (int v = 0; v < NWX_OF<KP>; ++v) {
            f += (fa[v].x + fa[v].y) + (fa[v].z + fa[v].w);
            fp += (fb[v].x + fb[v].y) + (fb[v].z + fb[v].w);
        }
        f += rx;
        fp += rxp;
        const bool acc = rv && fp <= f;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int c = c0 + 16 * q;
            const bool ok = rv && c < k;
            const float xa = acc ? xpq[q] : (ok ? xq[q] : 0.0f);
            sh.xat[c * GS + ri] = xa;
            sh.xs[ri][c] = xa;
            if (acc && c < k) a.X[(i0 + ri) * k + c] = xa;
        }
        if (c0 == 0 && rv) {
            a.alpha[i0 + ri] = acc ? al0 * a.step_up : al0 * a.step_down;
            rowreg_acc += acc ? rxp : rx;
            rej_acc += acc ? 0 : 1;
        }
    }
    lds_barrier();

    // ---- S6: column objective and Y gradient from the accepted rows -------------------
    XatFrag<KP, PREC> xa;
    xatfrag_load<KP, PREC>(xa, sh.xat, li, g);
    Frag<KP, PREC> xaf;
    frag_from_f32<KP, PREC>(xaf, &sh.xs[li][g * C]);
    xstep_s6<KP, TPW, PREC, LK>(a, apan, &sh.lt, sh.s_codes, sh.s_tcode, s_colw, yfr, xa, xaf, dyacc, hacc);
}

// Waves per SIMD the row pass is compiled for.  Narrow tables (few tiles per
// wavefront) run three workgroups per CU, which needs each wavefront within a
// third of the register file; the rest run one.
template <int KP, int TPW>
constexpr int XSTEP_MIN_WAVES = ((KP == 16 && TPW <= 4) || (KP == 32 && TPW <= 2)) ? 3 : 1;

template <int KP, int TPW, int PREC, int LK>
__global__ __launch_bounds__(NTX_OF<KP>, (XSTEP_MIN_WAVES<KP, TPW>)) void xstep_kernel(XStepArgs a)
{
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, g = lane >> 4;
    __shared__ XStepShared<KP, TPW, PREC> sh;
    // the panel buffers, LDS objects of their own
    __shared__ PanelBuf<KP, TPW, NWX_OF<KP>> sbuf0;
    __shared__ PanelBuf<KP, TPW, NWX_OF<KP>> sbuf1;
    __shared__ alignas(16) float s_colw[LK < 0 ? 16 * NWX_OF<KP> * TPW : 4];
    PanelBuf<KP, TPW, NWX_OF<KP>> *const pb0 = &sbuf0, *const pb1 = &sbuf1;
    const int nt = (int)(a.ldp / 16);
    const int64_t npanels = a.mp / 16;
    const int64_t G = gridDim.x;

    for (int j = threadIdx.x; j < a.ldp; j += NTX_OF<KP>) sh.s_codes[j] = a.codes[j];
    if constexpr (LK < 0) stage_colw(a.lt, 0, (int)a.ldp, a.ldp, s_colw, NTX_OF<KP>);
    if (threadIdx.x == 0) sh.lt = a.lt;
    __syncthreads();
    tile_codes(sh.s_codes, nt, sh.s_tcode, NTX_OF<KP>);
    // this wavefront's tiles of Y (fixed during the X half-step), resident in registers
    Frag<KP, PREC> yfr[TPW];
    YtFrag<KP, PREC> ytf[TPW];
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int t = min(w + NWX_OF<KP> * s, nt - 1);
        frag_load_y<KP, PREC>(yfr[s], a.ycur, 16 * t + li, g);
        ytfrag_load<KP, PREC>(ytf[s], a.ycur, a.ldp, 16 * t, li, g);
    }
    f32x4 dyacc[TPW][KP / 16];
#pragma unroll
    for (int s = 0; s < TPW; ++s)
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb) dyacc[s][kb] = f32x4{0.f, 0.f, 0.f, 0.f};
    float hacc[TPW];
#pragma unroll
    for (int s = 0; s < TPW; ++s) hacc[s] = 0.0f;
    float rowreg_acc = 0.0f;
    int rej_acc = 0;

    if (blockIdx.x < npanels)
        stage_panel<KP, TPW, NWX_OF<KP>, true>(*pb0, a.Ap, a.ldp, nt, a.X, a.m, a.k,
                                         a.alpha, blockIdx.x, w, lane);
    for (int64_t p = blockIdx.x; p < npanels; p += 2 * G) {
        const int64_t p1 = p + G, p2 = p + 2 * G;
        xstep_panel<KP, TPW, PREC, LK, 0>(a, sh, pb0, pb1, s_colw, p, p1 < npanels ? p1 : -1, yfr, ytf, dyacc,
                                          hacc, rowreg_acc, rej_acc);
        if (p1 < npanels)
            xstep_panel<KP, TPW, PREC, LK, 1>(a, sh, pb0, pb1, s_colw, p1, p2 < npanels ? p2 : -1, yfr, ytf, dyacc,
                                              hacc, rowreg_acc, rej_acc);
    }
    __syncthreads();

    // ---- this workgroup's partials ---------------------------------------------------
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int t = w + NWX_OF<KP> * s;
        if (t < nt) {
            const int64_t j0 = 16 * t;
#pragma unroll
            for (int kb = 0; kb < KP / 16; ++kb)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    a.part_dy[((int64_t)blockIdx.x * a.ldp + j0 + 4 * g + r) * KP + 16 * kb + li] =
                        GRAD_SCALE<LK> * dyacc[s][kb][r];
            // column j0 + li: the four lane groups' partials
            float h = hacc[s];
            h += __shfl_xor(h, 16, 64);
            h += __shfl_xor(h, 32, 64);
            if (g == 0) a.part_h[(int64_t)blockIdx.x * a.ldp + j0 + li] = h;
        }
    }
    // row regularizers and rejections live on the first lane of each row's sixteen
    float rr = sum_lanes<64>(rowreg_acc);
    int rj = (int)sum_lanes<64>((float)rej_acc);
    if (lane == 0) { sh.s_blk[w] = rr; sh.s_rej[w] = rj; }
    __syncthreads();
    if (threadIdx.x == 0) {
        float rsum = 0.0f;
        int jsum = 0;
#pragma unroll
        for (int v = 0; v < NWX_OF<KP>; ++v) { rsum += sh.s_blk[v]; jsum += sh.s_rej[v]; }
        a.part_rowreg[blockIdx.x] = rsum;
        a.part_rej[blockIdx.x] = jsum;
    }
}

// ---------------------------------------------------------------------------
// Y prox: reduce the partial gradients, step, prox (S7); remember h_j (old)
// ---------------------------------------------------------------------------
// A workgroup takes 64 consecutive (column, coordinate) elements; its four
// wavefronts each sum every fourth of the P partials (so the reads of a
// wavefront stay coalesced and the grid has n kp / 64 workgroups), and the
// first wavefront combines the four sums in a fixed order.
constexpr int YPROX_SPLIT = 4;
static_assert(YPROX_SPLIT == 4, "the combine below adds four sums");

template <int KP, int PREC>
__global__ __launch_bounds__(64 * YPROX_SPLIT) void yprox_kernel(YProxArgs a)
{
    __shared__ float s_part[YPROX_SPLIT][64];
    const int el = threadIdx.x & 63, ps = threadIdx.x >> 6;
    const int64_t t = (int64_t)blockIdx.x * 64 + el;
    const int64_t j = t / KP;
    const int c = (int)(t % KP);
    const bool valid = j < a.n;
    // the first wavefront's own inputs go out first, so that their latency
    // overlaps the partial loads: y, the step size, and its share of the
    // column-objective partials (the KP lanes of a column split them; summed
    // in a fixed order, then a butterfly identical in every lane)
    float y = 0.0f, al = 0.0f, h = 0.0f;
    if (ps == 0 && valid) {
        if (c < a.k) y = a.Y[j * a.k + c];
        al = a.alpha[j];
#pragma unroll 8
        for (int p = c; p < a.P; p += KP) h += a.part_h[(int64_t)p * a.ldp + j];
    }
    // fixed-order reduction of this wavefront's partials, eight running sums
    float gsum = 0.0f;
    if (valid) {
        const float *src = a.part_dy + j * KP + c;
        const int64_t stride = a.ldp * KP;
        float s8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        int p = ps;
        for (; p + 7 * YPROX_SPLIT < a.P; p += 8 * YPROX_SPLIT) {
#pragma unroll
            for (int q = 0; q < 8; ++q) s8[q] += src[(int64_t)(p + q * YPROX_SPLIT) * stride];
        }
        for (; p < a.P; p += YPROX_SPLIT) s8[0] += src[(int64_t)p * stride];
        gsum = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
    }
    s_part[ps][el] = gsum;
    __syncthreads();
    if (ps != 0) return;
    gsum = (s_part[0][el] + s_part[1][el]) + (s_part[2][el] + s_part[3][el]);
    const float yv = (valid && c < a.k) ? prox_elem(a.ry, al, y - al * gsum, c) : 0.0f;
    if (valid) {
        if (c < a.k) a.Yplus[j * a.k + c] = yv;
        if constexpr (PREC == P_FP32) {
            a.yplus.f32[j * KP + c] = yv;
        } else {
            __bf16 hi, lo;
            split_bf16(yv, hi, lo);
            a.yplus.hi[j * KP + c] = hi;
            a.yplus.lo[j * KP + c] = lo;
        }
    }
    float rc = (valid && c < a.k) ? reg_elem(a.ry, y, c) : 0.0f;
    float rcp = (valid && c < a.k) ? reg_elem_trial(a.ry, yv, c) : 0.0f;
    rc = sum_lanes<KP>(rc);
    rcp = sum_lanes<KP>(rcp);
    h = sum_lanes<KP>(h);
    if (valid && c == 0) {
        a.h_old[j] = h + rc;
        a.ry_plus[j] = rcp;
        a.ry_old[j] = rc;
    }
}

// ---------------------------------------------------------------------------
// pass 2: column objective at the trial Y+ (S8)
// ---------------------------------------------------------------------------
template <int KP, int TPW>
struct YCheckShared {
    PanelBuf<KP, TPW, NWY_OF<KP>> buf0, buf1;
    LossTab lt;
    uint8_t s_codes[16 * NWY_OF<KP> * TPW];
    int8_t s_tcode[NWY_OF<KP> * TPW];
};

template <int KP, int TPW, int PREC, int LK, int BUF>
__device__ __forceinline__ void ycheck_panel(const YCheckArgs a, YCheckShared<KP, TPW> &sh,
                                             const float *__restrict__ s_colw, int64_t p,
                                             int64_t p_next, int tile0, const Frag<KP, PREC> (&yfr)[TPW],
                                             f32x4 (&hacc)[TPW])
{
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, g = lane >> 4;
    constexpr int C = KP / 4;
    const int nt = (int)(a.ldp / 16);
    PanelBuf<KP, TPW, NWY_OF<KP>> &cur = BUF == 0 ? sh.buf0 : sh.buf1;
    PanelBuf<KP, TPW, NWY_OF<KP>> &nxt = BUF == 0 ? sh.buf1 : sh.buf0;
    const float4 *apan = cur.apan[w];
    const int64_t i0 = p * 16;

    wait_staged();
    // Everything this panel reads from LDS is read before the next panel's
    // direct-to-LDS loads go out (an LDS read issued after them would wait for
    // all of them): the X rows, straight from the staged block (16 x k,
    // contiguous), and the wavefront's table tiles.
    const int rows = (int)min<int64_t>(16, a.m - i0);
    Frag<KP, PREC> xf;
    {
        float xv[C];
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int c = g * C + q;
            xv[q] = (li < rows && c < a.k) ? cur.xrow[li * a.k + c] : 0.0f;
        }
        frag_from_f32<KP, PREC>(xf, xv);
    }
    float4 av[TPW];
#pragma unroll
    for (int s = 0; s < TPW; ++s) av[s] = tile_entries(apan, s, lane, tile0 + w + NWY_OF<KP> * s < nt);
    // no barrier until the next panel: the prefetch overlaps this panel's products
    if (p_next >= 0)
        stage_panel<KP, TPW, NWY_OF<KP>>(nxt, a.Ap, a.ldp, nt, a.X, a.m, a.k, nullptr, p_next, w, lane, tile0);
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        // the loss codes are staged per column block: index them by the tile's place in it
        const int tl = min(tile0 + w + NWY_OF<KP> * s, nt - 1) - tile0;
        const f32x4 zp = zprod<KP, PREC>(yfr[s], xf);
        float L4[4], G4[4];
        tile_loss<LK, false, false, TPW>(a.lu, sh.lt, sh.s_codes, sh.s_tcode, tl, zp, av[s], L4, G4, s_colw);
#pragma unroll
        for (int r = 0; r < 4; ++r) hacc[s][r] += L4[r];
    }
}

template <int KP, int TPW, int PREC, int LK>
__global__ __launch_bounds__(NTY_OF<KP>, 1) void ycheck_kernel(YCheckArgs a)
{
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, g = lane >> 4;
    __shared__ YCheckShared<KP, TPW> sh;
    __shared__ alignas(16) float s_colw[LK < 0 ? 16 * NWY_OF<KP> * TPW : 4];
    const int nt = (int)(a.ldp / 16);
    const int64_t npanels = a.mp / 16;
    // workgroup b takes column block b % ncb of the panels b / ncb, b / ncb + G, ...
    const int64_t G = gridDim.x / a.ncb;
    const int cb = (int)(blockIdx.x % a.ncb);
    const int64_t b0 = blockIdx.x / a.ncb;
    const int tile0 = cb * NWY_OF<KP> * TPW;

    // the loss codes of this workgroup's column block (columns past the table
    // repeat its last code, as the padding columns do)
    for (int j = threadIdx.x; j < 16 * NWY_OF<KP> * TPW; j += NTY_OF<KP>)
        sh.s_codes[j] = a.codes[min<int64_t>(16 * (int64_t)tile0 + j, a.ldp - 1)];
    if constexpr (LK < 0) stage_colw(a.lt, 16 * (int64_t)tile0, 16 * NWY_OF<KP> * TPW, a.ldp, s_colw, NTY_OF<KP>);
    if (threadIdx.x == 0) sh.lt = a.lt;
    __syncthreads();
    tile_codes(sh.s_codes, NWY_OF<KP> * TPW, sh.s_tcode, NTY_OF<KP>);
    Frag<KP, PREC> yfr[TPW];
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int t = min(tile0 + w + NWY_OF<KP> * s, nt - 1);
        frag_load_y<KP, PREC>(yfr[s], a.yplus, 16 * t + li, g);
    }
    f32x4 hacc[TPW];
#pragma unroll
    for (int s = 0; s < TPW; ++s) hacc[s] = f32x4{0.f, 0.f, 0.f, 0.f};

    if (b0 < npanels)
        stage_panel<KP, TPW, NWY_OF<KP>>(sh.buf0, a.Ap, a.ldp, nt, a.X, a.m, a.k, nullptr, b0, w, lane, tile0);
    for (int64_t p = b0; p < npanels; p += 2 * G) {
        const int64_t p1 = p + G, p2 = p + 2 * G;
        ycheck_panel<KP, TPW, PREC, LK, 0>(a, sh, s_colw, p, p1 < npanels ? p1 : -1, tile0, yfr, hacc);
        if (p1 < npanels)
            ycheck_panel<KP, TPW, PREC, LK, 1>(a, sh, s_colw, p1, p2 < npanels ? p2 : -1, tile0, yfr, hacc);
    }
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int t = tile0 + w + NWY_OF<KP> * s;
        if (t < nt) {
            const int64_t j0 = 16 * t;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float h = sum_lanes<16>(hacc[s][r]);
                if (li == 0) a.part_hp[b0 * a.ldp + j0 + 4 * g + r] = h;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// column decisions (S8), Y shadows for the next sweep, objective partials
// ---------------------------------------------------------------------------
template <int KP, int PREC>
__global__ __launch_bounds__(256) void yaccept_kernel(YAcceptArgs a)
{
    __shared__ double s_F[4];
    __shared__ int s_r[4];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = t / KP;
    const int c = (int)(t % KP);
    const bool valid = j < a.n;
    int acc = 0;
    double Fj = 0.0;
    int rj = 0;
    // every input goes out before the decision needs it: one round of loads
    float hp = 0.0f, ryp = 0.0f, h = 0.0f, al = 0.0f, yv = 0.0f;
    __bf16 yhi = to_bf16(0.0f), ylo = to_bf16(0.0f);
    if (valid) {
        ryp = a.ry_plus[j];
        h = a.h_old[j];
        if (c == 0) al = a.alpha[j];
        if (c < a.k) yv = a.Yplus[j * a.k + c];
        if constexpr (PREC != P_FP32) {
            yhi = a.yplus.hi[j * KP + c];
            if constexpr (PREC == P_BF16) ylo = a.yplus.lo[j * KP + c];
        }
        // the loads run ahead of the sum, which keeps the order of p
#pragma unroll 8
        for (int p = c; p < a.P; p += KP) hp += a.part_hp[(int64_t)p * a.ldp + j];
    }
    hp = sum_lanes<KP>(hp);   // the same value in every lane of the column
    if (a.phase == 1) {
        if (valid && c == 0) a.hpc[j] = hp + ryp;
        return;
    }
    if (valid) {
        hp += ryp;
        bool lead = true;     // the lane that counts the decision
        if (a.phase == 2) {
            // the block's sums, in column order (the same in every column of it)
            const int32_t b0 = a.blk0[j], b1 = a.blk1[j];
            float hb = 0.0f, hpb = 0.0f;
            for (int32_t e = b0; e < b1; ++e) {
                hb += a.h_old[e];
                hpb += a.hpc[e];
            }
            acc = hpb <= hb ? 1 : 0;
            lead = j == b0;
        } else {
            acc = hp <= h ? 1 : 0;
        }
        if (c == 0) {
            a.alpha[j] = acc ? al * a.step_up : al * a.step_down;
            Fj = acc ? (double)hp : (double)h;
            rj = (acc || !lead) ? 0 : 1;
        }
        if (acc) {
            if (c < a.k) a.Y[j * a.k + c] = yv;
            if constexpr (PREC == P_FP32) {
                a.ycur.f32[j * KP + c] = yv;
                a.ycur.t32[(int64_t)c * a.ldp + j] = yv;
            } else {
                a.ycur.hi[j * KP + c] = yhi;
                if constexpr (PREC == P_BF16) a.ycur.lo[j * KP + c] = ylo;
                a.ycur.tb[(int64_t)c * a.ldp + j] = yhi;
            }
        }
    }
    Fj = sum_lanes64<64>(Fj);
    rj = (int)sum_lanes<64>((float)rj);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { s_F[w] = Fj; s_r[w] = rj; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.part_F[blockIdx.x] = s_F[0] + s_F[1] + s_F[2] + s_F[3];
        a.part_rejc[blockIdx.x] = s_r[0] + s_r[1] + s_r[2] + s_r[3];
    }
}

// ---------------------------------------------------------------------------
// Y shadows from Y (fit start)
// ---------------------------------------------------------------------------
template <int KP, int PREC>
__global__ __launch_bounds__(256) void yshadow_kernel(YShadowArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = t / KP;
    const int c = (int)(t % KP);
    if (j >= a.ldp) return;
    const float yv = (j < a.n && c < a.k) ? a.Y[j * a.k + c] : 0.0f;
    if constexpr (PREC == P_FP32) {
        a.ys.f32[j * KP + c] = yv;
        a.ys.t32[(int64_t)c * a.ldp + j] = yv;
        if (a.yp.f32) a.yp.f32[j * KP + c] = 0.0f;
    } else {
        __bf16 hi, lo;
        split_bf16(yv, hi, lo);
        a.ys.hi[j * KP + c] = hi;
        if constexpr (PREC == P_BF16) a.ys.lo[j * KP + c] = lo;
        a.ys.tb[(int64_t)c * a.ldp + j] = hi;
        if (a.yp.hi) {
            a.yp.hi[j * KP + c] = to_bf16(0.0f);
            if constexpr (PREC == P_BF16) a.yp.lo[j * KP + c] = to_bf16(0.0f);
        }
    }
}

// ---------------------------------------------------------------------------
// objective and gradient (single pass, no decisions)
// ---------------------------------------------------------------------------
// grid: x = row chunks (persistent over 16-row panels), y = column blocks of
// NWX_OF<KP> * TPW tiles.  The structure of the fused row pass without the
// step: resident Y operands per wavefront, the panel's table tiles and X rows
// staged in LDS one panel ahead, and a barrier-free tile loop (restrict LDS
// operands) that the next panel's loads overlap.  A panel's dX partials are
// combined after the next panel's staging barrier, so each panel needs two
// barriers and the tile loop none.
template <int KP, int TPW, int PREC>
struct GradShared {
    float red_g[NWG_OF<KP>][16][RS<KP>];            // dX partials of the panel just computed
    LossTab lt;
    uint8_t s_codes[16 * NWG_OF<KP> * TPW];
    int8_t s_tcode[NWG_OF<KP> * TPW];
    double s_obj[NWG_OF<KP>];
};

template <int KP, int TPW, int PREC, int LK, bool WANT_GRAD>
__device__ __forceinline__ float grad_tiles(const LossGradArgs &a, PanelBuf<KP, TPW, NWG_OF<KP>> *__restrict__ nxt,
                                            int64_t p_next, const PanelBuf<KP, TPW, NWG_OF<KP>> *__restrict__ cur,
                                            int rows, int tile0, int nt, float *__restrict__ red_g,
                                            const LossTab *__restrict__ lt,
                                            const uint8_t *__restrict__ s_codes, const int8_t *__restrict__ s_tcode,
                                            const float *__restrict__ s_colw,
                                            const Frag<KP, PREC> (&yfr)[TPW], const YtFrag<KP, PREC> (&ytf)[TPW],
                                            f32x4 (&dyacc)[TPW][KP / 16])
{
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, g = lane >> 4;
    constexpr int C = KP / 4;
    const int k = a.k;
    // the panel's X rows straight from the staged block: row li (A operand of
    // z) and, for S6, rows 4g + q at coordinates 16 kb + li (B operand)
    Frag<KP, PREC> xf;
    {
        float xv[C];
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int c = g * C + q;
            xv[q] = (li < rows && c < k) ? cur->xrow[li * k + c] : 0.0f;
        }
        frag_from_f32<KP, PREC>(xf, xv);
    }
    XatFrag<KP, PREC> xa;
    if constexpr (WANT_GRAD) {
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb) {
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 4 * g + q, c = 16 * kb + li;
                v[q] = (i < rows && c < k) ? cur->xrow[i * k + c] : 0.0f;
            }
            if constexpr (PREC == P_FP32) xa.f[kb] = float4{v[0], v[1], v[2], v[3]};
            else xa.b[kb] = pack_bf16x4(v[0], v[1], v[2], v[3]);
        }
    }
    if (p_next >= 0)
        stage_panel<KP, TPW, NWG_OF<KP>>(*nxt, a.Ap, a.ldp, nt, a.X, a.m, a.k, nullptr, p_next, w, lane, tile0);
    const float4 *apan = cur->apan[w];
    float opart = 0.0f;
    f32x4 dx[KP / 16];
#pragma unroll
    for (int kb = 0; kb < KP / 16; ++kb) dx[kb] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 zn = zprod<KP, PREC>(yfr[0], xf);
    float4 an = apan[lane];
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int t = tile0 + w + NWG_OF<KP> * s;
        const f32x4 z = zn;
        const float4 av = an;
        if (s + 1 < TPW) {
            zn = zprod<KP, PREC>(yfr[s + 1], xf);
            an = apan[(s + 1) * 64 + lane];
        }
        if (t >= nt) continue;
        float L4[4], G[4];
        tile_loss<LK, WANT_GRAD, false, TPW>(a.lu, *lt, s_codes, s_tcode, t - tile0, z, av, L4, G, s_colw);
        opart += (L4[0] + L4[1]) + (L4[2] + L4[3]);
        if constexpr (WANT_GRAD) {
            s3_resident<KP, PREC>(dx, G, ytf[s]);
            float gT[4];
            transpose_g(G, gT);
            s6_resident<KP, PREC>(dyacc[s], gT, xa);
        }
    }
    if constexpr (WANT_GRAD) {
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb)
#pragma unroll
            for (int r = 0; r < 4; ++r) red_g[(w * 16 + 4 * g + r) * RS<KP> + 16 * kb + li] = dx[kb][r];
    }
    return opart;
}

// dX rows of panel p from the wavefronts' partials (after a barrier).
template <int KP, int LK>
__device__ __forceinline__ void grad_reduce_dx(const LossGradArgs &a, const float (*red_g)[16][RS<KP>], int64_t p)
{
    const int64_t i0 = p * 16;
    for (int t = threadIdx.x; t < 16 * KP; t += NTG_OF<KP>) {
        const int i = t / KP, c = t % KP;
        if (i0 + i < a.m && c < a.k) {
            float s = 0.0f;
#pragma unroll
            for (int q = 0; q < NWG_OF<KP>; ++q) s += red_g[q][i][c];
            s *= GRAD_SCALE<LK>;
            if (a.part_dx) a.part_dx[((int64_t)blockIdx.y * a.m + i0 + i) * a.k + c] = s;
            else a.dX[(i0 + i) * a.k + c] = s;
        }
    }
}

template <int KP, int TPW, int PREC, int LK, bool WANT_GRAD>
__global__ __launch_bounds__(NTG_OF<KP>, 1) void lossgrad_kernel(LossGradArgs a)
{
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, g = lane >> 4;
    __shared__ GradShared<KP, TPW, PREC> sh;
    // the panel buffers, LDS objects of their own: the compiler then tells the
    // next panel's direct-to-LDS loads apart from the tile loop's LDS traffic
    // and keeps them in flight through it
    __shared__ PanelBuf<KP, TPW, NWG_OF<KP>> sbuf0;
    __shared__ PanelBuf<KP, TPW, NWG_OF<KP>> sbuf1;
    __shared__ alignas(16) float s_colw[LK < 0 ? 16 * NWG_OF<KP> * TPW : 4];
    const int nt = (int)(a.ldp / 16);
    const int64_t npanels = a.mp / 16;
    const int64_t G = gridDim.x;
    const int tile0 = (int)blockIdx.y * NWG_OF<KP> * TPW;
    const int ntb = min(NWG_OF<KP> * TPW, nt - tile0);   // tiles of this column block

    for (int j = threadIdx.x; j < 16 * NWG_OF<KP> * TPW; j += NTG_OF<KP>)
        sh.s_codes[j] = a.codes[min(16 * tile0 + j, (int)a.ldp - 1)];
    if constexpr (LK < 0) stage_colw(a.lt, 16 * (int64_t)tile0, 16 * NWG_OF<KP> * TPW, a.ldp, s_colw, NTG_OF<KP>);
    if (threadIdx.x == 0) sh.lt = a.lt;
    __syncthreads();
    tile_codes(sh.s_codes, ntb, sh.s_tcode, NTG_OF<KP>);
    Frag<KP, PREC> yfr[TPW];
    YtFrag<KP, PREC> ytf[TPW];
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int t = min(tile0 + w + NWG_OF<KP> * s, nt - 1);
        frag_load_y<KP, PREC>(yfr[s], a.ycur, 16 * t + li, g);
        if constexpr (WANT_GRAD) ytfrag_load<KP, PREC>(ytf[s], a.ycur, a.ldp, 16 * t, li, g);
    }
    f32x4 dyacc[TPW][KP / 16];
#pragma unroll
    for (int s = 0; s < TPW; ++s)
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb) dyacc[s][kb] = f32x4{0.f, 0.f, 0.f, 0.f};
    double obj = 0.0;

    if (blockIdx.x < npanels)
        stage_panel<KP, TPW, NWG_OF<KP>>(sbuf0, a.Ap, a.ldp, nt, a.X, a.m, a.k, nullptr, blockIdx.x, w, lane,
                                         tile0);
    int64_t prev = -1;
    for (int64_t p = blockIdx.x; p < npanels; p += 2 * G) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t pc = p + b * G;
            if (pc >= npanels) break;
            const int64_t pn = pc + G < npanels ? pc + G : -1;
            PanelBuf<KP, TPW, NWG_OF<KP>> &cur = b == 0 ? sbuf0 : sbuf1;
            PanelBuf<KP, TPW, NWG_OF<KP>> &nxt = b == 0 ? sbuf1 : sbuf0;
            wait_staged();
            if (WANT_GRAD && prev >= 0) grad_reduce_dx<KP, LK>(a, sh.red_g, prev);
            // orders the reads of red_g above before this panel's writes; an
            // LDS-only barrier, so the stores of the reduced rows stay in flight
            // through the tile loop instead of being waited for here
            lds_barrier();
            const int rows = (int)min<int64_t>(16, a.m - pc * 16);
            obj += (double)grad_tiles<KP, TPW, PREC, LK, WANT_GRAD>(a, &nxt, pn, &cur, rows, tile0, nt, &sh.red_g[0][0][0],
                                                                    &sh.lt, sh.s_codes, sh.s_tcode,
                                                                    s_colw, yfr, ytf, dyacc);
            prev = pc;
        }
    }
    __syncthreads();
    if (WANT_GRAD && prev >= 0) grad_reduce_dx<KP, LK>(a, sh.red_g, prev);
    if constexpr (WANT_GRAD) {
#pragma unroll
        for (int s = 0; s < TPW; ++s) {
            const int t = tile0 + w + NWG_OF<KP> * s;
            if (t < nt && w + NWG_OF<KP> * s < NWG_OF<KP> * TPW) {
                const int64_t j0 = 16 * t;
#pragma unroll
                for (int kb = 0; kb < KP / 16; ++kb)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        a.part_dy[((int64_t)blockIdx.x * a.ldp + j0 + 4 * g + r) * KP + 16 * kb + li] =
                            GRAD_SCALE<LK> * dyacc[s][kb][r];
            }
        }
    }
    obj = sum_lanes64<64>(obj);
    if (lane == 0) sh.s_obj[w] = obj;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < NWG_OF<KP>; ++q) s += sh.s_obj[q];
        a.part_obj[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// the row half-step in column blocks (tables wider than the fused row pass
// holds, whose wavefronts keep every tile of a row's Y operands resident)
// ---------------------------------------------------------------------------
// Three passes over the table on a grid of row chunks x column blocks of
// NWX_OF<KP> * TPW tiles, as the gradient pass:
//   MODE 0  at X: each row's loss sum and gradient over the block (S1-S3)
//   MODE 1  at the trial rows X+: each row's loss sum over the block (S5)
//   MODE 2  at the decided rows: each column's loss sum and Y-gradient
//           partial over the workgroup's rows (S6)
// with the row steps (S4) and the decisions between them, in dense.hip.  The
// sums over column blocks are taken there, in block order.
template <int KP, int TPW, int MODE>
struct WideShared {
    float red_g[MODE == 0 ? NWX_OF<KP> : 1][16][RS<KP>];   // MODE 0: dX partials of the panel
    float red_f[NWX_OF<KP>][16];           // MODE 0, 1: row loss partials of the panel
    LossTab lt;
    uint8_t s_codes[16 * NWX_OF<KP> * TPW];
    int8_t s_tcode[NWX_OF<KP> * TPW];
};

template <int KP, int TPW, int PREC, int LK, int MODE>
__device__ __forceinline__ void xwide_tiles(const XWideArgs &a, PanelBuf<KP, TPW, NWX_OF<KP>> *__restrict__ nxt,
                                            int64_t p_next, const PanelBuf<KP, TPW, NWX_OF<KP>> *__restrict__ cur,
                                            int rows, int tile0, int nt, float *__restrict__ red_g,
                                            float *__restrict__ red_f, const LossTab *__restrict__ lt,
                                            const uint8_t *__restrict__ s_codes, const int8_t *__restrict__ s_tcode,
                                            const float *__restrict__ s_colw,
                                            const Frag<KP, PREC> (&yfr)[TPW], const YtFrag<KP, PREC> (&ytf)[TPW],
                                            f32x4 (&dyacc)[TPW][KP / 16], float (&hacc)[TPW])
{
    constexpr bool SWZ = MODE == 2;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, g = lane >> 4;
    constexpr int C = KP / 4;
    const int k = a.k;
    // row li's coordinates g C .. g C + C - 1: the A operand of z in MODE 2,
    // the B operand otherwise
    Frag<KP, PREC> xf;
    {
        float xv[C];
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int c = g * C + q;
            xv[q] = (li < rows && c < k) ? cur->xrow[li * k + c] : 0.0f;
        }
        frag_from_f32<KP, PREC>(xf, xv);
    }
    XatFrag<KP, PREC> xa;   // MODE 2: rows 4g + q at coordinates 16 kb + li (B operand of dY)
    if constexpr (MODE == 2) {
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb) {
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 4 * g + q, c = 16 * kb + li;
                v[q] = (i < rows && c < k) ? cur->xrow[i * k + c] : 0.0f;
            }
            if constexpr (PREC == P_FP32) xa.f[kb] = float4{v[0], v[1], v[2], v[3]};
            else xa.b[kb] = pack_bf16x4(v[0], v[1], v[2], v[3]);
        }
    }
    if (p_next >= 0)
        stage_panel<KP, TPW, NWX_OF<KP>, SWZ>(*nxt, a.Ap, a.ldp, nt, a.X, a.m, a.k, nullptr, p_next, w, lane, tile0);
    const float4 *apan = cur->apan[w];
    float opart = 0.0f;
    f32x4 dx[KP / 16];
#pragma unroll
    for (int kb = 0; kb < KP / 16; ++kb) dx[kb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // software pipelined as the fused row pass
    f32x4 zn = MODE == 2 ? zprod<KP, PREC>(xf, yfr[0]) : zprod<KP, PREC>(yfr[0], xf);
    float4 an = MODE == 2 ? tile_entries_t(apan, 0, li, g) : apan[lane];
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int t = tile0 + w + NWX_OF<KP> * s;
        const f32x4 z = zn;
        const float4 av = an;
        if (s + 1 < TPW) {
            zn = MODE == 2 ? zprod<KP, PREC>(xf, yfr[s + 1]) : zprod<KP, PREC>(yfr[s + 1], xf);
            an = MODE == 2 ? tile_entries_t(apan, s + 1, li, g) : apan[(s + 1) * 64 + lane];
        }
        if (t >= nt) continue;
        float L4[4], G[4];
        tile_loss<LK, MODE != 1, MODE == 2, TPW>(a.lu, *lt, s_codes, s_tcode, t - tile0, z, av, L4, G, s_colw);
        const float l4 = (L4[0] + L4[1]) + (L4[2] + L4[3]);
        if constexpr (MODE == 2) {
            hacc[s] += l4;
            s6_resident<KP, PREC>(dyacc[s], G, xa);
        } else {
            opart += l4;
            if constexpr (MODE == 0) s3_resident<KP, PREC>(dx, G, ytf[s]);
        }
    }
    if constexpr (MODE != 2) {
        // row li: the four lane groups' partials (the same sum in every lane)
        opart += __shfl_xor(opart, 16, 64);
        opart += __shfl_xor(opart, 32, 64);
        if (g == 0) red_f[w * 16 + li] = opart;
    }
    if constexpr (MODE == 0) {
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb)
#pragma unroll
            for (int r = 0; r < 4; ++r) red_g[(w * 16 + 4 * g + r) * RS<KP> + 16 * kb + li] = dx[kb][r];
    }
}

// Panel p's rows (modes 0, 1): the wavefronts' partials in wavefront order.
template <int KP, int LK, int MODE, typename SH>
__device__ __forceinline__ void xwide_reduce_rows(const XWideArgs &a, const SH &sh, int64_t p, int cb)
{
    const int64_t i0 = p * 16;
    const int rows = (int)min<int64_t>(16, a.m - i0);
    if (threadIdx.x < 16 && threadIdx.x < rows) {
        float f = 0.0f;
#pragma unroll
        for (int v = 0; v < NWX_OF<KP>; ++v) f += sh.red_f[v][threadIdx.x];
        a.part_f[(int64_t)cb * a.mp + i0 + threadIdx.x] = f;
    }
    if constexpr (MODE == 0) {
        for (int t = threadIdx.x; t < 16 * KP; t += NTX_OF<KP>) {
            const int i = t / KP, c = t % KP;
            if (i < rows && c < a.k) {
                float s = 0.0f;
#pragma unroll
                for (int v = 0; v < NWX_OF<KP>; ++v) s += sh.red_g[v][i][c];
                a.part_dx[((int64_t)cb * a.m + i0 + i) * a.k + c] = GRAD_SCALE<LK> * s;
            }
        }
    }
}

template <int KP, int TPW, int PREC, int LK, int MODE>
__global__ __launch_bounds__(NTX_OF<KP>, 1) void xwide_kernel(XWideArgs a)
{
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, g = lane >> 4;
    constexpr bool SWZ = MODE == 2;
    __shared__ WideShared<KP, TPW, MODE> sh;
    __shared__ alignas(16) float s_colw[LK < 0 ? 16 * NWX_OF<KP> * TPW : 4];
    // the panel buffers, LDS objects of their own (as in the fused row pass)
    __shared__ PanelBuf<KP, TPW, NWX_OF<KP>> sbuf0;
    __shared__ PanelBuf<KP, TPW, NWX_OF<KP>> sbuf1;
    const int nt = (int)(a.ldp / 16);
    const int64_t npanels = a.mp / 16;
    const int64_t G = gridDim.x;
    const int cb = (int)blockIdx.y;
    const int tile0 = cb * NWX_OF<KP> * TPW;
    const int ntb = min(NWX_OF<KP> * TPW, nt - tile0);   // tiles of this column block

    for (int j = threadIdx.x; j < 16 * NWX_OF<KP> * TPW; j += NTX_OF<KP>)
        sh.s_codes[j] = a.codes[min<int64_t>(16 * (int64_t)tile0 + j, a.ldp - 1)];
    if constexpr (LK < 0) stage_colw(a.lt, 16 * (int64_t)tile0, 16 * NWX_OF<KP> * TPW, a.ldp, s_colw, NTX_OF<KP>);
    if (threadIdx.x == 0) sh.lt = a.lt;
    __syncthreads();
    tile_codes(sh.s_codes, ntb, sh.s_tcode, NTX_OF<KP>);
    Frag<KP, PREC> yfr[TPW];
    YtFrag<KP, PREC> ytf[TPW];
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int t = min(tile0 + w + NWX_OF<KP> * s, nt - 1);
        frag_load_y<KP, PREC>(yfr[s], a.ycur, 16 * t + li, g);
        if constexpr (MODE == 0) ytfrag_load<KP, PREC>(ytf[s], a.ycur, a.ldp, 16 * t, li, g);
    }
    f32x4 dyacc[TPW][KP / 16];
    float hacc[TPW];
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        hacc[s] = 0.0f;
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb) dyacc[s][kb] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

    if (blockIdx.x < npanels)
        stage_panel<KP, TPW, NWX_OF<KP>, SWZ>(sbuf0, a.Ap, a.ldp, nt, a.X, a.m, a.k, nullptr, blockIdx.x, w, lane,
                                              tile0);
    int64_t prev = -1;
    for (int64_t p = blockIdx.x; p < npanels; p += 2 * G) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t pc = p + b * G;
            if (pc >= npanels) break;
            const int64_t pn = pc + G < npanels ? pc + G : -1;
            PanelBuf<KP, TPW, NWX_OF<KP>> &cur = b == 0 ? sbuf0 : sbuf1;
            PanelBuf<KP, TPW, NWX_OF<KP>> &nxt = b == 0 ? sbuf1 : sbuf0;
            wait_staged();
            // the previous panel's rows, reduced here so that their stores stay
            // in flight through this panel's tile loop
            if constexpr (MODE != 2) {
                if (prev >= 0) xwide_reduce_rows<KP, LK, MODE>(a, sh, prev, cb);
                lds_barrier();
            }
            const int64_t i0 = pc * 16;
            const int rows = (int)min<int64_t>(16, a.m - i0);
            xwide_tiles<KP, TPW, PREC, LK, MODE>(a, &nxt, pn, &cur, rows, tile0, nt, &sh.red_g[0][0][0],
                                                 &sh.red_f[0][0], &sh.lt, sh.s_codes, sh.s_tcode, s_colw, yfr, ytf,
                                                 dyacc, hacc);
            prev = pc;
        }
    }
    if constexpr (MODE != 2) {
        __syncthreads();
        if (prev >= 0) xwide_reduce_rows<KP, LK, MODE>(a, sh, prev, cb);
    }
    if constexpr (MODE == 2) {
#pragma unroll
        for (int s = 0; s < TPW; ++s) {
            const int t = tile0 + w + NWX_OF<KP> * s;
            if (t < nt) {
                const int64_t j0 = 16 * t;
#pragma unroll
                for (int kb = 0; kb < KP / 16; ++kb)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        a.part_dy[((int64_t)blockIdx.x * a.ldp + j0 + 4 * g + r) * KP + 16 * kb + li] =
                            GRAD_SCALE<LK> * dyacc[s][kb][r];
                // column j0 + li: the four lane groups' partials
                float h = hacc[s];
                h += __shfl_xor(h, 16, 64);
                h += __shfl_xor(h, 32, 64);
                if (g == 0) a.part_h[(int64_t)blockIdx.x * a.ldp + j0 + li] = h;
            }
        }
    }
}

// dY = sum over row chunks of the partials; dX = sum over column blocks.
template <int KP>
__global__ __launch_bounds__(256) void reduce_dy_kernel(ReduceArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = t / KP;
    const int c = (int)(t % KP);
    if (j >= a.n || c >= a.k) return;
    float s = 0.0f;
    for (int p = 0; p < a.P; ++p) s += a.part_dy[((int64_t)p * a.ldp + j) * KP + c];
    a.dY[j * a.k + c] = s;
}

}  // namespace glrm
