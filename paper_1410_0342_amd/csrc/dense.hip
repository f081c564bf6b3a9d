// Dense-layout kernels of the GLRM sweep for gfx950.
//
// The table sits in the workspace as a padded copy (rows to a multiple of 16,
// columns to a multiple of 16) in which every unobserved entry is a quiet NaN,
// so one 4-byte load gives both the value and the observation bit.
//
// Work decomposition: a workgroup of 8 wavefronts walks 16-row panels.  The
// panel's columns are cut into 16-wide tiles and tile t belongs to wavefront
// t mod 8 for the whole launch, so each wavefront can keep per-column
// accumulators (column objective, Y gradient) in registers across panels.
//
// Matrix-core products per 16 x 16 tile (i = row of the panel, j = column):
//   z     Z^T(16j x 16i) = Y_tile(16j x kp) . X_panel^T        -> lane holds z(i=l%16, j=4(l/16)+r)
//   S3    dX(16i x 16kc) += G(16i x 16j) . Y_tile(16j x 16kc)   (G straight from the z layout)
//   S6    dY(16j x 16kc) += G^T(16j x 16i) . X(16i x 16kc)      (G transposed through LDS)
// The k index each lane feeds is a free choice as long as both operands use
// the same one: lane group g = l/16 feeds the contiguous run k = g*kp/4 ...
// (g+1)*kp/4 - 1, which makes every operand load one contiguous vector.
#include "glrm_device.h"
#include "glrm_kernels.h"

namespace glrm {

constexpr int NW = 8;            // wavefronts per workgroup
constexpr int NT = NW * 64;      // threads per workgroup
constexpr int GS = 20;           // row stride (floats) of the per-wave transpose tile

// ---------------------------------------------------------------------------
// operand fragments
// ---------------------------------------------------------------------------
template <int KP, int PREC>
struct Frag {
    static constexpr int C = KP / 4;      // values per lane
    float f[PREC == P_FP32 ? C : 1];
    __bf16 hi[PREC == P_FP32 ? 1 : C];
    __bf16 lo[PREC == P_BF16 ? C : 1];
};

// From fp32 values (LDS panel row or registers).
template <int KP, int PREC>
__device__ __forceinline__ void frag_from_f32(Frag<KP, PREC> &fr, const float *src)
{
#pragma unroll
    for (int q = 0; q < KP / 4; ++q) {
        float v = src[q];
        if constexpr (PREC == P_FP32) fr.f[q] = v;
        else if constexpr (PREC == P_BF16) split_bf16(v, fr.hi[q], fr.lo[q]);
        else fr.hi[q] = to_bf16(v);
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
        // C bf16 = 2C bytes: 8, 16 or 32
        const __bf16 *ph = ys.hi + j * KP + g * C;
        if constexpr (C == 4) {
            *reinterpret_cast<uint2 *>(fr.hi) = *reinterpret_cast<const uint2 *>(ph);
        } else {
#pragma unroll
            for (int q = 0; q < C / 8; ++q)
                reinterpret_cast<uint4 *>(fr.hi)[q] = reinterpret_cast<const uint4 *>(ph)[q];
        }
        if constexpr (PREC == P_BF16) {
            const __bf16 *pl = ys.lo + j * KP + g * C;
            if constexpr (C == 4) {
                *reinterpret_cast<uint2 *>(fr.lo) = *reinterpret_cast<const uint2 *>(pl);
            } else {
#pragma unroll
                for (int q = 0; q < C / 8; ++q)
                    reinterpret_cast<uint4 *>(fr.lo)[q] = reinterpret_cast<const uint4 *>(pl)[q];
            }
        }
    }
}

__device__ __forceinline__ f32x4 mfma_bf16_4(const __bf16 *a, const __bf16 *b, f32x4 acc)
{
    i16x4 av, bv;
#pragma unroll
    for (int s = 0; s < 4; ++s) { av[s] = bf16_bits(a[s]); bv[s] = bf16_bits(b[s]); }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma_bf16_8(const __bf16 *a, const __bf16 *b, f32x4 acc)
{
    bf16x8 av, bv;
#pragma unroll
    for (int s = 0; s < 8; ++s) { av[s] = a[s]; bv[s] = b[s]; }
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
}

template <int KP>
__device__ __forceinline__ f32x4 mfma_run(const __bf16 *a, const __bf16 *b, f32x4 acc)
{
    if constexpr (KP == 16) return mfma_bf16_4(a, b, acc);
    else {
#pragma unroll
        for (int q = 0; q < KP / 32; ++q) acc = mfma_bf16_8(a + 8 * q, b + 8 * q, acc);
        return acc;
    }
}

// Z^T tile = Y_tile . X_panel^T.  Split bf16: the two small cross terms first.
template <int KP, int PREC>
__device__ __forceinline__ f32x4 zprod(const Frag<KP, PREC> &y, const Frag<KP, PREC> &x)
{
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    if constexpr (PREC == P_FP32) {
#pragma unroll
        for (int q = 0; q < KP / 4; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(y.f[q], x.f[q], acc, 0, 0, 0);
    } else {
        if constexpr (PREC == P_BF16) {
            acc = mfma_run<KP>(y.lo, x.hi, acc);
            acc = mfma_run<KP>(y.hi, x.lo, acc);
        }
        acc = mfma_run<KP>(y.hi, x.hi, acc);
    }
    return acc;
}

// S3: dX block kb (16 rows x 16 of k) += G(16i x 16j) . Y_tile(16j x 16kc).
// G[r] = G(i = l%16, j = 4g + r).  Y^T shadow row kc holds y_j for all j.
template <int KP, int PREC>
__device__ __forceinline__ void s3_accum(f32x4 (&dx)[KP / 16], const float (&G)[4], const YShadow &ys,
                                         int64_t ldp, int64_t j0, int li, int g)
{
#pragma unroll
    for (int kb = 0; kb < KP / 16; ++kb) {
        const int64_t off = (int64_t)(16 * kb + li) * ldp + j0 + 4 * g;
        if constexpr (PREC == P_FP32) {
            float4 b = *reinterpret_cast<const float4 *>(ys.t32 + off);
            dx[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(G[0], b.x, dx[kb], 0, 0, 0);
            dx[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(G[1], b.y, dx[kb], 0, 0, 0);
            dx[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(G[2], b.z, dx[kb], 0, 0, 0);
            dx[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(G[3], b.w, dx[kb], 0, 0, 0);
        } else {
            i16x4 av, bv;
            *reinterpret_cast<uint2 *>(&bv) = *reinterpret_cast<const uint2 *>(ys.tb + off);
#pragma unroll
            for (int s = 0; s < 4; ++s) av[s] = bf16_bits(to_bf16(G[s]));
            dx[kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, dx[kb], 0, 0, 0);
        }
    }
}

// S6: dY block (16 j x 16 kc) += G^T(16j x 16i) . X(16i x 16kc).  gT[s] =
// G(i = 4g + s, j = l%16); xat is the panel's X transposed in LDS ([kc][i]).
template <int KP, int PREC>
__device__ __forceinline__ void s6_accum(f32x4 (&dy)[KP / 16], const float (&gT)[4], const float *xat, int li, int g)
{
#pragma unroll
    for (int kb = 0; kb < KP / 16; ++kb) {
        float4 b = *reinterpret_cast<const float4 *>(xat + (16 * kb + li) * GS + 4 * g);
        if constexpr (PREC == P_FP32) {
            dy[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(gT[0], b.x, dy[kb], 0, 0, 0);
            dy[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(gT[1], b.y, dy[kb], 0, 0, 0);
            dy[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(gT[2], b.z, dy[kb], 0, 0, 0);
            dy[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(gT[3], b.w, dy[kb], 0, 0, 0);
        } else {
            i16x4 av, bv;
#pragma unroll
            for (int s = 0; s < 4; ++s) av[s] = bf16_bits(to_bf16(gT[s]));
            bv[0] = bf16_bits(to_bf16(b.x)); bv[1] = bf16_bits(to_bf16(b.y));
            bv[2] = bf16_bits(to_bf16(b.z)); bv[3] = bf16_bits(to_bf16(b.w));
            dy[kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, dy[kb], 0, 0, 0);
        }
    }
}

// Transpose the wave's 16x16 G tile through LDS.
__device__ __forceinline__ void transpose_g(float *gsc, const float (&G)[4], float (&gT)[4], int li, int g)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) gsc[(4 * g + r) * GS + li] = G[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float4 v = *reinterpret_cast<const float4 *>(gsc + li * GS + 4 * g);
    gT[0] = v.x; gT[1] = v.y; gT[2] = v.z; gT[3] = v.w;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Loss codes of the lane's four columns.
__device__ __forceinline__ void load_codes(const uint8_t *codes, int64_t j, int (&cd)[4])
{
    uchar4 c = *reinterpret_cast<const uchar4 *>(codes + j);
    cd[0] = c.x; cd[1] = c.y; cd[2] = c.z; cd[3] = c.w;
}

__device__ __forceinline__ void entry_lg(const LossTab &lt, int code, float u, float a, float &l, float &gr)
{
    const int q = lt.uniform >= 0 ? lt.uniform : code;
    loss_lg(lt.kind[q], lt.levels[q], lt.param[q], u, a, l, gr);
}

__device__ __forceinline__ float entry_l(const LossTab &lt, int code, float u, float a)
{
    const int q = lt.uniform >= 0 ? lt.uniform : code;
    return loss_l(lt.kind[q], lt.levels[q], lt.param[q], u, a);
}

// Load the 16 x k panel of a factor into LDS as fp32 [16][KP] (zero padded).
template <int KP>
__device__ __forceinline__ void load_panel(float (*xs)[KP], const float *X, int64_t i0, int64_t m, int k)
{
    for (int t = threadIdx.x; t < 16 * KP; t += NT) {
        const int i = t / KP, c = t % KP;
        const int64_t gi = i0 + i;
        xs[i][c] = (gi < m && c < k) ? X[gi * k + c] : 0.0f;
    }
}

// ---------------------------------------------------------------------------
// pass 1: fused X half-step (S1-S5) + Y-gradient and column-objective partials (S6)
// ---------------------------------------------------------------------------
template <int KP, int TPW, int PREC>
__global__ __launch_bounds__(NT, 1) void xstep_kernel(XStepArgs a)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    constexpr int C = KP / 4;

    __shared__ float xs[16][KP];
    __shared__ float xp[16][KP];
    __shared__ __attribute__((aligned(16))) float xat[KP * GS];
    __shared__ float red_f[NW][16];
    __shared__ float red_g[NW][16][KP + 1];
    __shared__ __attribute__((aligned(16))) float gsc_all[NW][16 * GS];
    __shared__ float s_f[16], s_rx[16], s_rxp[16];
    __shared__ int s_acc[16];
    __shared__ float s_blk[NW];
    __shared__ int s_rej[NW];
    __shared__ float s_h[16 * NW * TPW];
    __shared__ float4 apan_all[NW][TPW * 64];   // each wavefront's A tiles, [tile][lane]
    float4 *apan = apan_all[w];

    float *gsc = gsc_all[w];
    const int64_t ntiles = a.ldp / 16;
    const int64_t npanels = a.mp / 16;

    f32x4 dyacc[TPW][KP / 16];
#pragma unroll
    for (int s = 0; s < TPW; ++s)
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb) dyacc[s][kb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // column objective partials of this workgroup; column tiles are owned by
    // one wavefront, so the updates never collide
    for (int64_t j = threadIdx.x; j < a.ldp; j += NT) s_h[j] = 0.0f;
    float rowreg_acc = 0.0f;   // sum of r over accepted rows (thread-strided, reduced at the end)
    int rej_acc = 0;

    for (int64_t p = blockIdx.x; p < npanels; p += gridDim.x) {
        const int64_t i0 = p * 16;
        load_panel<KP>(xs, a.X, i0, a.m, a.k);
        __syncthreads();

        // ---- S1-S3: z, loss, derivative, row objective, row gradient ---------
        Frag<KP, PREC> xf;
        frag_from_f32<KP, PREC>(xf, &xs[li][g * C]);
        float fpart = 0.0f;
        f32x4 dx[KP / 16];
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb) dx[kb] = f32x4{0.f, 0.f, 0.f, 0.f};
        {
            // all of this wavefront's table loads in flight at once, then staged in LDS
            // tiles past the last one re-load the last tile (in bounds, never used)
            const float *arow = a.Ap + (i0 + li) * a.ldp + 4 * g;
            const int nt = (int)ntiles;
            float4 areg[TPW];
#pragma unroll
            for (int s = 0; s < TPW; ++s) {
                const int t = min(w + NW * s, nt - 1);
                areg[s] = *reinterpret_cast<const float4 *>(arow + 16 * t);
            }
#pragma unroll
            for (int s = 0; s < TPW; ++s) apan[s * 64 + lane] = areg[s];
        }
#pragma unroll 2
        for (int s = 0; s < TPW; ++s) {
            const int64_t t = w + NW * s;
            if (t < ntiles) {
                const int64_t j0 = 16 * t;
                const float4 av = apan[s * 64 + lane];
                Frag<KP, PREC> yf;
                frag_load_y<KP, PREC>(yf, a.ycur, j0 + li, g);
                const f32x4 z = zprod<KP, PREC>(yf, xf);
                int cd[4];
                load_codes(a.codes, j0 + 4 * g, cd);
                float G[4];
                const float avr[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float l = 0.f, gr = 0.f;
                    if (avr[r] == avr[r]) entry_lg(a.lt, cd[r], z[r], avr[r], l, gr);
                    fpart += l;
                    G[r] = gr;
                }
                s3_accum<KP, PREC>(dx, G, a.ycur, a.ldp, j0, li, g);
            }
        }
        fpart += __shfl_xor(fpart, 16, 64);
        fpart += __shfl_xor(fpart, 32, 64);
        if (g == 0) red_f[w][li] = fpart;
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb)
#pragma unroll
            for (int r = 0; r < 4; ++r) red_g[w][4 * g + r][16 * kb + li] = dx[kb][r];
        __syncthreads();

        // ---- S4: prox step, regularizer values -------------------------------
        for (int t = threadIdx.x; t < 16 * KP; t += NT) {
            const int i = t / KP, c = t % KP;
            const int64_t gi = i0 + i;
            float gs = 0.0f;
#pragma unroll
            for (int q = 0; q < NW; ++q) gs += red_g[q][i][c];
            const float x = xs[i][c];
            const float al = gi < a.m ? a.alpha[gi] : 0.0f;
            const float xv = (c < a.k) ? prox_elem(a.rx, al, x - al * gs) : 0.0f;
            xp[i][c] = xv;
            float rc = c < a.k ? reg_elem(a.rx, x) : 0.0f;
            float rcp = c < a.k ? reg_elem(a.rx, xv) : 0.0f;
            rc = sum_lanes<KP>(rc);
            rcp = sum_lanes<KP>(rcp);
            if (c == 0) {
                float f = 0.0f;
#pragma unroll
                for (int q = 0; q < NW; ++q) f += red_f[q][i];
                s_f[i] = f + rc;
                s_rx[i] = rc;
                s_rxp[i] = rcp;
            }
        }
        __syncthreads();

        // ---- S5: row objective at the trial point -----------------------------
        Frag<KP, PREC> xpf;
        frag_from_f32<KP, PREC>(xpf, &xp[li][g * C]);
        float fppart = 0.0f;
#pragma unroll 2
        for (int s = 0; s < TPW; ++s) {
            const int64_t t = w + NW * s;
            if (t < ntiles) {
                const int64_t j0 = 16 * t;
                Frag<KP, PREC> yf;
                frag_load_y<KP, PREC>(yf, a.ycur, j0 + li, g);
                const f32x4 zp = zprod<KP, PREC>(yf, xpf);
                int cd[4];
                load_codes(a.codes, j0 + 4 * g, cd);
                const float4 av = apan[s * 64 + lane];
                const float avr[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (avr[r] == avr[r]) fppart += entry_l(a.lt, cd[r], zp[r], avr[r]);
            }
        }
        fppart += __shfl_xor(fppart, 16, 64);
        fppart += __shfl_xor(fppart, 32, 64);
        if (g == 0) red_f[w][li] = fppart;
        __syncthreads();

        // ---- decision per row ----------------------------------------------------
        if (threadIdx.x < 16) {
            const int i = threadIdx.x;
            const int64_t gi = i0 + i;
            int acc = 0;
            if (gi < a.m) {
                float fp = 0.0f;
#pragma unroll
                for (int q = 0; q < NW; ++q) fp += red_f[q][i];
                fp += s_rxp[i];
                acc = (fp <= s_f[i]) ? 1 : 0;
                const float al = a.alpha[gi];
                a.alpha[gi] = acc ? al * a.step_up : al * a.step_down;
                rowreg_acc += acc ? s_rxp[i] : s_rx[i];
                rej_acc += acc ? 0 : 1;
            }
            s_acc[i] = acc;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < 16 * KP; t += NT) {
            const int i = t / KP, c = t % KP;
            const int64_t gi = i0 + i;
            const float xa = s_acc[i] ? xp[i][c] : xs[i][c];
            xat[c * GS + i] = xa;
            xs[i][c] = xa;
            if (s_acc[i] && c < a.k) a.X[gi * a.k + c] = xa;
        }
        __syncthreads();

        // ---- S6: column objective and Y gradient from the accepted rows ----------
        Frag<KP, PREC> xaf;
        frag_from_f32<KP, PREC>(xaf, &xs[li][g * C]);
#pragma unroll
        for (int s = 0; s < TPW; ++s) {
            const int64_t t = w + NW * s;
            if (t < ntiles) {
                const int64_t j0 = 16 * t;
                Frag<KP, PREC> yf;
                frag_load_y<KP, PREC>(yf, a.ycur, j0 + li, g);
                const f32x4 zs = zprod<KP, PREC>(yf, xaf);
                int cd[4];
                load_codes(a.codes, j0 + 4 * g, cd);
                const float4 av = apan[s * 64 + lane];
                const float avr[4] = {av.x, av.y, av.z, av.w};
                float G[4], gT[4], hl[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float l = 0.f, gr = 0.f;
                    if (avr[r] == avr[r]) entry_lg(a.lt, cd[r], zs[r], avr[r], l, gr);
                    hl[r] = sum_lanes<16>(l);
                    G[r] = gr;
                }
                if (li == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) s_h[j0 + 4 * g + r] += hl[r];
                }
                transpose_g(gsc, G, gT, li, g);
                s6_accum<KP, PREC>(dyacc[s], gT, xat, li, g);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
    }

    // ---- write this workgroup's partials ---------------------------------------
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int64_t t = w + NW * s;
        if (t < ntiles) {
            const int64_t j0 = 16 * t;
#pragma unroll
            for (int kb = 0; kb < KP / 16; ++kb)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    a.part_dy[((int64_t)blockIdx.x * a.ldp + j0 + 4 * g + r) * KP + 16 * kb + li] = dyacc[s][kb][r];
        }
    }
    for (int64_t j = threadIdx.x; j < a.ldp; j += NT) a.part_h[(int64_t)blockIdx.x * a.ldp + j] = s_h[j];
    // rowreg / rejects live on threads 0..15 of wave 0
    float rr = sum_lanes<64>(rowreg_acc);
    int rj = (int)sum_lanes<64>((float)rej_acc);
    if (lane == 0) { s_blk[w] = rr; s_rej[w] = rj; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.part_rowreg[blockIdx.x] = s_blk[0];
        a.part_rej[blockIdx.x] = s_rej[0];
    }
}

// ---------------------------------------------------------------------------
// Y prox: reduce the partial gradients, step, prox (S7); remember h_j (old)
// ---------------------------------------------------------------------------
template <int KP, int PREC>
__global__ __launch_bounds__(256) void yprox_kernel(YProxArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = t / KP;
    const int c = (int)(t % KP);
    const bool valid = j < a.n;
    float gsum = 0.0f;
    if (valid)
        for (int p = 0; p < a.P; ++p) gsum += a.part_dy[((int64_t)p * a.ldp + j) * KP + c];
    const float y = (valid && c < a.k) ? a.Y[j * a.k + c] : 0.0f;
    const float al = valid ? a.alpha[j] : 0.0f;
    const float yv = (valid && c < a.k) ? prox_elem(a.ry, al, y - al * gsum) : 0.0f;
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
    float rc = (valid && c < a.k) ? reg_elem(a.ry, y) : 0.0f;
    float rcp = (valid && c < a.k) ? reg_elem(a.ry, yv) : 0.0f;
    rc = sum_lanes<KP>(rc);
    rcp = sum_lanes<KP>(rcp);
    if (valid && c == 0) {
        float h = 0.0f;
        for (int p = 0; p < a.P; ++p) h += a.part_h[(int64_t)p * a.ldp + j];
        a.h_old[j] = h + rc;
        a.ry_plus[j] = rcp;
        a.ry_old[j] = rc;
    }
}

// ---------------------------------------------------------------------------
// pass 2: column objective at the trial Y+ (S8)
// ---------------------------------------------------------------------------
template <int KP, int TPW, int PREC>
__global__ __launch_bounds__(NT, 1) void ycheck_kernel(YCheckArgs a)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    constexpr int C = KP / 4;
    __shared__ float xs[16][KP];
    const int64_t ntiles = a.ldp / 16;
    const int64_t npanels = a.mp / 16;

    f32x4 hacc[TPW];
#pragma unroll
    for (int s = 0; s < TPW; ++s) hacc[s] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int64_t p = blockIdx.x; p < npanels; p += gridDim.x) {
        const int64_t i0 = p * 16;
        load_panel<KP>(xs, a.X, i0, a.m, a.k);
        __syncthreads();
        Frag<KP, PREC> xf;
        frag_from_f32<KP, PREC>(xf, &xs[li][g * C]);
#pragma unroll
        for (int s = 0; s < TPW; ++s) {
            const int64_t t = w + NW * s;
            if (t < ntiles) {
                const int64_t j0 = 16 * t;
                const float4 av = *reinterpret_cast<const float4 *>(a.Ap + (i0 + li) * a.ldp + j0 + 4 * g);
                Frag<KP, PREC> yf;
                frag_load_y<KP, PREC>(yf, a.yplus, j0 + li, g);
                const f32x4 zp = zprod<KP, PREC>(yf, xf);
                int cd[4];
                load_codes(a.codes, j0 + 4 * g, cd);
                const float avr[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (avr[r] == avr[r]) hacc[s][r] += entry_l(a.lt, cd[r], zp[r], avr[r]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
        const int64_t t = w + NW * s;
        if (t < ntiles) {
            const int64_t j0 = 16 * t;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float h = sum_lanes<16>(hacc[s][r]);
                if (li == 0) a.part_hp[(int64_t)blockIdx.x * a.ldp + j0 + 4 * g + r] = h;
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
    if (valid) {
        float hp = 0.0f;
        for (int p = 0; p < a.P; ++p) hp += a.part_hp[(int64_t)p * a.ldp + j];
        hp += a.ry_plus[j];
        const float h = a.h_old[j];
        acc = hp <= h ? 1 : 0;
        if (c == 0) {
            const float al = a.alpha[j];
            a.alpha[j] = acc ? al * a.step_up : al * a.step_down;
            Fj = acc ? (double)hp : (double)h;
            rj = acc ? 0 : 1;
        }
        if (acc) {
            const float yv = c < a.k ? a.Yplus[j * a.k + c] : 0.0f;
            if (c < a.k) a.Y[j * a.k + c] = yv;
            if constexpr (PREC == P_FP32) {
                a.ycur.f32[j * KP + c] = yv;
                a.ycur.t32[(int64_t)c * a.ldp + j] = yv;
            } else {
                a.ycur.hi[j * KP + c] = a.yplus.hi[j * KP + c];
                if constexpr (PREC == P_BF16) a.ycur.lo[j * KP + c] = a.yplus.lo[j * KP + c];
                a.ycur.tb[(int64_t)c * a.ldp + j] = a.yplus.hi[j * KP + c];
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
// grid: x = row chunks, y = column blocks of NW*TPW tiles
template <int KP, int TPW, int PREC, bool WANT_GRAD>
__global__ __launch_bounds__(NT, 1) void lossgrad_kernel(LossGradArgs a)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    constexpr int C = KP / 4;
    __shared__ float xs[16][KP];
    __shared__ __attribute__((aligned(16))) float xat[KP * GS];
    __shared__ float red_g[NW][16][KP + 1];
    __shared__ __attribute__((aligned(16))) float gsc_all[NW][16 * GS];
    __shared__ double s_obj[NW];
    float *gsc = gsc_all[w];
    const int64_t ntiles = a.ldp / 16;
    const int64_t npanels = a.mp / 16;
    const int64_t tile0 = (int64_t)blockIdx.y * NW * TPW;

    f32x4 dyacc[TPW][KP / 16];
#pragma unroll
    for (int s = 0; s < TPW; ++s)
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb) dyacc[s][kb] = f32x4{0.f, 0.f, 0.f, 0.f};
    double obj = 0.0;

    for (int64_t p = blockIdx.x; p < npanels; p += gridDim.x) {
        const int64_t i0 = p * 16;
        load_panel<KP>(xs, a.X, i0, a.m, a.k);
        if (WANT_GRAD) {
            for (int t = threadIdx.x; t < 16 * KP; t += NT) {
                const int i = t / KP, c = t % KP;
                xat[c * GS + i] = (i0 + i < a.m && c < a.k) ? a.X[(i0 + i) * a.k + c] : 0.0f;
            }
        }
        __syncthreads();
        Frag<KP, PREC> xf;
        frag_from_f32<KP, PREC>(xf, &xs[li][g * C]);
        f32x4 dx[KP / 16];
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb) dx[kb] = f32x4{0.f, 0.f, 0.f, 0.f};
        float opart = 0.0f;
#pragma unroll
        for (int s = 0; s < TPW; ++s) {
            const int64_t t = tile0 + w + NW * s;
            if (t < ntiles) {
                const int64_t j0 = 16 * t;
                const float4 av = *reinterpret_cast<const float4 *>(a.Ap + (i0 + li) * a.ldp + j0 + 4 * g);
                Frag<KP, PREC> yf;
                frag_load_y<KP, PREC>(yf, a.ycur, j0 + li, g);
                const f32x4 z = zprod<KP, PREC>(yf, xf);
                int cd[4];
                load_codes(a.codes, j0 + 4 * g, cd);
                const float avr[4] = {av.x, av.y, av.z, av.w};
                float G[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float l = 0.f, gr = 0.f;
                    if (avr[r] == avr[r]) {
                        if (WANT_GRAD) entry_lg(a.lt, cd[r], z[r], avr[r], l, gr);
                        else l = entry_l(a.lt, cd[r], z[r], avr[r]);
                    }
                    opart += l;
                    G[r] = gr;
                }
                if (WANT_GRAD) {
                    s3_accum<KP, PREC>(dx, G, a.ycur, a.ldp, j0, li, g);
                    float gT[4];
                    transpose_g(gsc, G, gT, li, g);
                    s6_accum<KP, PREC>(dyacc[s], gT, xat, li, g);
                }
            }
        }
        obj += (double)opart;
        if (WANT_GRAD) {
#pragma unroll
            for (int kb = 0; kb < KP / 16; ++kb)
#pragma unroll
                for (int r = 0; r < 4; ++r) red_g[w][4 * g + r][16 * kb + li] = dx[kb][r];
            __syncthreads();
            for (int t = threadIdx.x; t < 16 * KP; t += NT) {
                const int i = t / KP, c = t % KP;
                if (i0 + i < a.m && c < a.k) {
                    float s = 0.0f;
#pragma unroll
                    for (int q = 0; q < NW; ++q) s += red_g[q][i][c];
                    if (a.part_dx) a.part_dx[((int64_t)blockIdx.y * a.m + i0 + i) * a.k + c] = s;
                    else a.dX[(i0 + i) * a.k + c] = s;
                }
            }
        }
        __syncthreads();
    }
    if (WANT_GRAD) {
#pragma unroll
        for (int s = 0; s < TPW; ++s) {
            const int64_t t = tile0 + w + NW * s;
            if (t < ntiles) {
                const int64_t j0 = 16 * t;
#pragma unroll
                for (int kb = 0; kb < KP / 16; ++kb)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        a.part_dy[((int64_t)blockIdx.x * a.ldp + j0 + 4 * g + r) * KP + 16 * kb + li] = dyacc[s][kb][r];
            }
        }
    }
    obj = sum_lanes64<64>(obj);
    if (lane == 0) s_obj[w] = obj;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < NW; ++q) s += s_obj[q];
        a.part_obj[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
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

__global__ __launch_bounds__(256) void reduce_dx_kernel(ReduceArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= a.m * a.k) return;
    float s = 0.0f;
    for (int b = 0; b < a.CB; ++b) s += a.part_dx[(int64_t)b * a.m * a.k + t];
    a.dX[t] = s;
}

// FP64 objective: z in double from the fp32 factors, loss in double.
__global__ __launch_bounds__(256) void objective64_kernel(Obj64Args a)
{
    __shared__ double xsd[16][GLRM_MAXK_DEV + 1];
    __shared__ double ysd[64][GLRM_MAXK_DEV + 1];
    __shared__ double sred[4];
    const int64_t ntile_j = (a.ldp + 63) / 64;
    const int64_t npanels = a.mp / 16;
    double acc = 0.0;
    for (int64_t blk = blockIdx.x; blk < npanels * ntile_j; blk += gridDim.x) {
        const int64_t p = blk / ntile_j, jt = blk % ntile_j;
        const int64_t i0 = p * 16, j0 = jt * 64;
        for (int t = threadIdx.x; t < 16 * a.k; t += 256) {
            const int i = t / a.k, c = t % a.k;
            xsd[i][c] = i0 + i < a.m ? (double)a.X[(i0 + i) * a.k + c] : 0.0;
        }
        for (int t = threadIdx.x; t < 64 * a.k; t += 256) {
            const int jj = t / a.k, c = t % a.k;
            ysd[jj][c] = j0 + jj < a.n ? (double)a.Y[(j0 + jj) * a.k + c] : 0.0;
        }
        __syncthreads();
        const int jj = threadIdx.x & 63;
        const int64_t j = j0 + jj;
        if (j < a.n) {
            const int code = a.codes[j];
            const int q = a.lt.uniform >= 0 ? a.lt.uniform : code;
            for (int ii = threadIdx.x >> 6; ii < 16; ii += 4) {
                const int64_t i = i0 + ii;
                if (i >= a.m) break;
                const float av = a.Ap[i * a.ldp + j];
                if (av == av) {
                    double z = 0.0;
                    for (int c = 0; c < a.k; ++c) z += xsd[ii][c] * ysd[jj][c];
                    acc += loss_l64(a.lt.kind[q], a.lt.levels[q], (double)a.lt.param[q], z, (double)av);
                }
            }
        }
        __syncthreads();
    }
    acc = sum_lanes64<64>(acc);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) a.part_obj[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define GLRM_DISPATCH_KP(KPV, ...)                                    \
    switch (KPV) {                                                    \
    case 16: { constexpr int KP = 16; __VA_ARGS__; } break;           \
    case 32: { constexpr int KP = 32; __VA_ARGS__; } break;           \
    case 64: { constexpr int KP = 64; __VA_ARGS__; } break;           \
    default: return hipErrorInvalidValue;                              \
    }
#define GLRM_DISPATCH_PREC(PV, ...)                                   \
    switch (PV) {                                                     \
    case P_FP32: { constexpr int PREC = P_FP32; __VA_ARGS__; } break; \
    case P_BF16: { constexpr int PREC = P_BF16; __VA_ARGS__; } break; \
    case P_BF16_PLAIN: { constexpr int PREC = P_BF16_PLAIN; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                              \
    }
#define GLRM_DISPATCH_TPW(TV, ...)                                    \
    switch (TV) {                                                     \
    case 1: { constexpr int TPW = 1; __VA_ARGS__; } break;            \
    case 2: { constexpr int TPW = 2; __VA_ARGS__; } break;            \
    case 4: { constexpr int TPW = 4; __VA_ARGS__; } break;            \
    case 8: { constexpr int TPW = 8; __VA_ARGS__; } break;            \
    default: return hipErrorInvalidValue;                              \
    }

hipError_t launch_xstep(const XStepArgs &a, int kp, int tpw, int prec, int grid, hipStream_t st)
{
    GLRM_DISPATCH_PREC(prec, GLRM_DISPATCH_KP(kp, GLRM_DISPATCH_TPW(tpw,
        if constexpr (KP == 64 && TPW == 8) return hipErrorInvalidValue;
        else hipLaunchKernelGGL((xstep_kernel<KP, TPW, PREC>), dim3(grid), dim3(NT), 0, st, a))));
    return hipGetLastError();
}

hipError_t launch_ycheck(const YCheckArgs &a, int kp, int tpw, int prec, int grid, hipStream_t st)
{
    GLRM_DISPATCH_PREC(prec, GLRM_DISPATCH_KP(kp, GLRM_DISPATCH_TPW(tpw,
        hipLaunchKernelGGL((ycheck_kernel<KP, TPW, PREC>), dim3(grid), dim3(NT), 0, st, a))));
    return hipGetLastError();
}

hipError_t launch_yprox(const YProxArgs &a, int kp, int prec, hipStream_t st)
{
    const int64_t threads = a.n * (int64_t)kp;
    const int blocks = (int)((threads + 255) / 256);
    GLRM_DISPATCH_PREC(prec, GLRM_DISPATCH_KP(kp,
        hipLaunchKernelGGL((yprox_kernel<KP, PREC>), dim3(blocks), dim3(256), 0, st, a)));
    return hipGetLastError();
}

hipError_t launch_yaccept(const YAcceptArgs &a, int kp, int prec, int blocks, hipStream_t st)
{
    GLRM_DISPATCH_PREC(prec, GLRM_DISPATCH_KP(kp,
        hipLaunchKernelGGL((yaccept_kernel<KP, PREC>), dim3(blocks), dim3(256), 0, st, a)));
    return hipGetLastError();
}

int yaccept_blocks(int64_t n, int kp) { return (int)((n * kp + 255) / 256); }

hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_yshadow(const YShadowArgs &a, int kp, int prec, hipStream_t st)
{
    const int64_t threads = a.ldp * (int64_t)kp;
    const int blocks = (int)((threads + 255) / 256);
    GLRM_DISPATCH_PREC(prec, GLRM_DISPATCH_KP(kp,
        hipLaunchKernelGGL((yshadow_kernel<KP, PREC>), dim3(blocks), dim3(256), 0, st, a)));
    return hipGetLastError();
}

hipError_t launch_lossgrad(const LossGradArgs &a, int kp, int tpw, int prec, bool want_grad, int gx, int gy,
                           hipStream_t st)
{
    if (want_grad) {
        GLRM_DISPATCH_PREC(prec, GLRM_DISPATCH_KP(kp, GLRM_DISPATCH_TPW(tpw,
            if constexpr (KP == 64 && TPW == 8) return hipErrorInvalidValue;
            else hipLaunchKernelGGL((lossgrad_kernel<KP, TPW, PREC, true>), dim3(gx, gy), dim3(NT), 0, st, a))));
    } else {
        GLRM_DISPATCH_PREC(prec, GLRM_DISPATCH_KP(kp, GLRM_DISPATCH_TPW(tpw,
            hipLaunchKernelGGL((lossgrad_kernel<KP, TPW, PREC, false>), dim3(gx, gy), dim3(NT), 0, st, a))));
    }
    return hipGetLastError();
}

hipError_t launch_reduce_dy(const ReduceArgs &a, int kp, hipStream_t st)
{
    const int blocks = (int)((a.n * (int64_t)kp + 255) / 256);
    GLRM_DISPATCH_KP(kp, hipLaunchKernelGGL((reduce_dy_kernel<KP>), dim3(blocks), dim3(256), 0, st, a));
    return hipGetLastError();
}

hipError_t launch_reduce_dx(const ReduceArgs &a, hipStream_t st)
{
    const int blocks = (int)((a.m * (int64_t)a.k + 255) / 256);
    hipLaunchKernelGGL(reduce_dx_kernel, dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_objective64(const Obj64Args &a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(objective64_kernel, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace glrm
