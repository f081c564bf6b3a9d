// Device-side building blocks of the GLRM sweep on gfx950: losses, their
// derivatives, regularizers, proximal operators, bfloat16 splitting, the
// matrix-core fragment products and wavefront reductions.
//
// Losses: Section 4 (quadratic eq. qpca, Huber), Section 5.2 (hinge, logistic,
// ordinal hinge eq. ord-pca).  Regularizers: Section 3.  Proximal operators:
// definition in Section 7.2.  At a kink the derivative takes the
// strict-inequality branch (the kink contributes 0).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace glrm {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) short i16x4;

enum { L_QUAD = 0, L_HUBER = 1, L_LOGISTIC = 2, L_HINGE = 3, L_ORDINAL = 4, L_CATEGORICAL = 5, L_MORDINAL = 6 };
enum { R_ZERO = 0, R_QUAD = 1, R_L1 = 2, R_NONNEG = 3 };
enum { P_FP32 = 0, P_BF16 = 1, P_FP64 = 2, P_BF16_PLAIN = 3 };

constexpr int MAX_LOSSES = 16;

// Loss table handed to kernels by value.
struct LossTab {
    int32_t kind[MAX_LOSSES];
    int32_t levels[MAX_LOSSES];
    float param[MAX_LOSSES];
    int32_t n;
    int32_t uniform;   // >= 0: every column uses losses[uniform] with weight 1; -1: per-column table
    const float *colw; // per-column loss weights (padded to the table's width), or null for 1
};

// A regularizer; `offset` marks coordinate 0 as the model's offset
// (Section 3.3): 1 = held at the constant 1 (the rows of X), 2 = free and
// unpenalized (the columns of Y); 0 = no offset.
struct Reg {
    int32_t kind;
    float w;
    int32_t offset;
};

// ---- losses ------------------------------------------------------------------

// Ordinal hinge in closed form.  The lower hinges (1 - u + a')_+ for
// a' = 1..a-1 are positive exactly for a' > u - 1, i.e. from lo = max(1, floor u);
// the upper hinges (1 + u - a')_+ for a' = a+1..d are positive exactly for
// a' < u + 1, i.e. up to hi = min(d, ceil u).  Each positive run is an
// arithmetic series; every bound stays in floating point.
template <typename T>
__device__ __forceinline__ void ordinal_loss(T u, T a, int d, T &l, T &g, bool want_g)
{
    const T lo = fmax(T(1), floor(u));
    const T hi = fmin(T(d), ceil(u));
    const T n1 = fmax(T(0), a - lo);     // lower hinges in [lo, a - 1]
    const T n2 = fmax(T(0), hi - a);     // upper hinges in [a + 1, hi]
    const T s1 = n1 * ((lo + a - T(1)) * T(0.5) - (u - T(1)));
    const T s2 = n2 * ((u + T(1)) - (a + T(1) + hi) * T(0.5));
    l = s1 + s2;
    if (want_g) g = n2 - n1;
}

// exp(-|t|) with the hardware base-2 exponential (about 1 ulp; it flushes to 0
// below 2^-126, where the logistic loss and its derivative no longer need it).
__device__ __forceinline__ float exp_neg_abs(float t)
{
    return __builtin_amdgcn_exp2f(-fabsf(t) * 1.4426950408889634f);
}

// log(1 + e) for e in [0, 1], from log(1 + e) = 2 artanh(s), s = e / (2 + e):
// s <= 1/3, so the odd series 2 (s + s^3/3 + ... + s^13/13) is within
// 2 s^15 / (15 (1 - s^2)) of it, below 2e-8 relative.  Exact at e = 0, and
// accurate for tiny e, where 1 + e rounds to 1.
__device__ __forceinline__ float log1p_unit(float e)
{
    const float s = e * __builtin_amdgcn_rcpf(2.0f + e);
    const float s2 = s * s;
    float p = 1.0f / 13.0f;
    p = p * s2 + 1.0f / 11.0f;
    p = p * s2 + 1.0f / 9.0f;
    p = p * s2 + 1.0f / 7.0f;
    p = p * s2 + 1.0f / 5.0f;
    p = p * s2 + 1.0f / 3.0f;
    p = p * s2 + 1.0f;
    return 2.0f * s * p;
}

// Loss value and derivative in u, float, for a loss kind known at compile time.
template <int K>
__device__ __forceinline__ void loss_lg_k(int levels, float param, float u, float a, float &l, float &g)
{
    if constexpr (K == L_QUAD) {
        const float d = u - a;
        l = d * d;
        g = 2.0f * d;
    } else if constexpr (K == L_HUBER) {
        const float r = u - a, ar = fabsf(r);
        if (ar <= param) { l = 0.5f * r * r; g = r; }
        else { l = param * ar - 0.5f * param * param; g = r > 0.0f ? param : -param; }
    } else if constexpr (K == L_LOGISTIC) {
        // t = -a u;  l = max(t,0) + log1p(exp(-|t|));  dl/du = -a sigmoid(t)
        const float t = -a * u;
        const float e = exp_neg_abs(t);
        const float inv = __builtin_amdgcn_rcpf(1.0f + e);
        l = fmaxf(t, 0.0f) + log1p_unit(e);
        g = -a * (t >= 0.0f ? inv : e * inv);
    } else if constexpr (K == L_HINGE) {
        // written so that a NaN product gives a NaN loss (never a zero one)
        const float au = a * u;
        if (!(au >= 1.0f)) { l = 1.0f - au; g = -a; }
        else { l = 0.0f; g = 0.0f; }
    } else {
        ordinal_loss<float>(u, a, levels, l, g, true);
    }
}

template <int K>
__device__ __forceinline__ float loss_l_k(int levels, float param, float u, float a)
{
    if constexpr (K == L_QUAD) {
        const float d = u - a;
        return d * d;
    } else if constexpr (K == L_HUBER) {
        const float r = u - a, ar = fabsf(r);
        return ar <= param ? 0.5f * r * r : param * ar - 0.5f * param * param;
    } else if constexpr (K == L_LOGISTIC) {
        const float t = -a * u;
        return fmaxf(t, 0.0f) + log1p_unit(exp_neg_abs(t));
    } else if constexpr (K == L_HINGE) {
        const float au = a * u;
        return !(au >= 1.0f) ? 1.0f - au : 0.0f;
    } else {
        float l, g;
        ordinal_loss<float>(u, a, levels, l, g, false);
        return l;
    }
}

// The same with the kind chosen at run time.
__device__ __forceinline__ void loss_lg(int kind, int levels, float param, float u, float a, float &l, float &g)
{
    switch (kind) {
    case L_QUAD: loss_lg_k<L_QUAD>(levels, param, u, a, l, g); break;
    case L_HUBER: loss_lg_k<L_HUBER>(levels, param, u, a, l, g); break;
    case L_LOGISTIC: loss_lg_k<L_LOGISTIC>(levels, param, u, a, l, g); break;
    case L_HINGE: loss_lg_k<L_HINGE>(levels, param, u, a, l, g); break;
    default: loss_lg_k<L_ORDINAL>(levels, param, u, a, l, g); break;
    }
}

__device__ __forceinline__ float loss_l(int kind, int levels, float param, float u, float a)
{
    switch (kind) {
    case L_QUAD: return loss_l_k<L_QUAD>(levels, param, u, a);
    case L_HUBER: return loss_l_k<L_HUBER>(levels, param, u, a);
    case L_LOGISTIC: return loss_l_k<L_LOGISTIC>(levels, param, u, a);
    case L_HINGE: return loss_l_k<L_HINGE>(levels, param, u, a);
    default: return loss_l_k<L_ORDINAL>(levels, param, u, a);
    }
}

// Double precision loss value (final objective check).
__device__ __forceinline__ double loss_l64(int kind, int levels, double param, double u, double a)
{
    switch (kind) {
    case L_QUAD: {
        double d = u - a;
        return d * d;
    }
    case L_HUBER: {
        double r = u - a, ar = fabs(r);
        return ar <= param ? 0.5 * r * r : param * ar - 0.5 * param * param;
    }
    case L_LOGISTIC: {
        double t = -a * u;
        return fmax(t, 0.0) + log1p(exp(-fabs(t)));
    }
    case L_HINGE: {
        double au = a * u;
        return !(au >= 1.0) ? 1.0 - au : 0.0;
    }
    default: {
        double l, g;
        ordinal_loss<double>(u, a, levels, l, g, false);
        return l;
    }
    }
}

// Double precision loss derivative, with the same choice at each kink as the
// float form (the strict-inequality branch).
__device__ __forceinline__ double loss_g64(int kind, int levels, double param, double u, double a)
{
    switch (kind) {
    case L_QUAD: return 2.0 * (u - a);
    case L_HUBER: {
        const double r = u - a;
        return fabs(r) <= param ? r : (r > 0.0 ? param : -param);
    }
    case L_LOGISTIC: return -a / (1.0 + exp(a * u));
    case L_HINGE: return !(a * u >= 1.0) ? -a : 0.0;
    default: {
        double l, g;
        ordinal_loss<double>(u, a, levels, l, g, true);
        return g;
    }
    }
}

// ---- regularizers -------------------------------------------------------------

// One coordinate's share of r(x) (the sum over coordinates is r); c is the
// coordinate.  With an offset, coordinate 0 carries no penalty, and on the
// rows of X only x_0 = 1 is feasible.
__device__ __forceinline__ float reg_elem(const Reg &r, float x, int c)
{
    if (c == 0 && r.offset) return (r.offset == 1 && x != 1.0f) ? __builtin_huge_valf() : 0.0f;
    switch (r.kind) {
    case R_QUAD: return r.w * x * x;
    case R_L1: return r.w * fabsf(x);
    case R_NONNEG: return x < 0.0f ? __builtin_huge_valf() : 0.0f;
    default: return 0.0f;
    }
}

__device__ __forceinline__ double reg_elem64(const Reg &r, double x, int c)
{
    if (c == 0 && r.offset) return (r.offset == 1 && x != 1.0) ? __builtin_huge_val() : 0.0;
    switch (r.kind) {
    case R_QUAD: return (double)r.w * x * x;
    case R_L1: return (double)r.w * fabs(x);
    case R_NONNEG: return x < 0.0 ? __builtin_huge_val() : 0.0;
    default: return 0.0;
    }
}

// A trial point's share of r(x) with the step gate folded in: r(x) plus
// 0 * x, which is exactly r(x) for a finite coordinate and NaN for an
// infinite or NaN one, so a trial objective built from it is NaN and the
// step is rejected (a non-finite point lies outside the model's domain).
__device__ __forceinline__ float reg_elem_trial(const Reg &r, float x, int c)
{
    return reg_elem(r, x, c) + 0.0f * x;
}

// One coordinate of the least-magnitude subgradient of r at x: the projection
// of 0 onto the coordinate's interval of subgradients (quadratic 2 w x; l1
// w sign x, the interval [-w, w] at 0; nonnegative 0 inside the orthant and on
// its boundary); NaN outside r's domain, where no subgradient exists.
__device__ __forceinline__ float reg_grad_elem(const Reg &r, float x, int c)
{
    const float qnan = __builtin_nanf("");
    if (c == 0 && r.offset) return (r.offset == 1 && x != 1.0f) ? qnan : 0.0f;
    switch (r.kind) {
    case R_QUAD: return 2.0f * r.w * x;
    case R_L1: return x > 0.0f ? r.w : (x < 0.0f ? -r.w : 0.0f);
    case R_NONNEG: return x < 0.0f ? qnan : 0.0f;
    default: return 0.0f;
    }
}

// prox_{alpha r}(v), coordinate-wise (every supported r is separable); the
// offset coordinate is projected onto 1 (X) or left as it is (Y).
__device__ __forceinline__ float prox_elem(const Reg &r, float alpha, float v, int c)
{
    if (c == 0 && r.offset) return r.offset == 1 ? 1.0f : v;
    switch (r.kind) {
    case R_QUAD: return v / (1.0f + 2.0f * alpha * r.w);
    case R_L1: {
        float t = fabsf(v) - alpha * r.w;
        return t > 0.0f ? copysignf(t, v) : 0.0f;
    }
    case R_NONNEG: return v > 0.0f ? v : 0.0f;
    default: return v;
    }
}

// ---- bfloat16 ----------------------------------------------------------------

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }
__device__ __forceinline__ float from_bf16(__bf16 x) { return (float)x; }

// x = hi + lo + O(2^-16 |x|): the two-term split used for z.
__device__ __forceinline__ void split_bf16(float x, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

__device__ __forceinline__ short bf16_bits(__bf16 x) { return __builtin_bit_cast(short, x); }

// Four values to bf16 (round to nearest even), packed as one matrix-core operand.
__device__ __forceinline__ i16x4 pack_bf16x4(float a, float b, float c, float d)
{
    typedef __attribute__((ext_vector_type(2))) float f32x2;
    typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
    const bf16x2 p0 = __builtin_convertvector((f32x2){a, b}, bf16x2);
    const bf16x2 p1 = __builtin_convertvector((f32x2){c, d}, bf16x2);
    const uint2 u = {__builtin_bit_cast(uint32_t, p0), __builtin_bit_cast(uint32_t, p1)};
    return __builtin_bit_cast(i16x4, u);
}

// ---- workgroup barrier for LDS traffic ---------------------------------------

// Barrier that orders LDS accesses only: this wavefront's LDS operations
// complete (lgkmcnt), then s_barrier.  Outstanding global loads, including
// direct-to-LDS loads into a buffer that nobody reads before the next full
// barrier, stay in flight; __syncthreads() would drain them.  The signal
// fences keep the compiler from moving memory accesses across the barrier.
__device__ __forceinline__ void lds_barrier()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0); vmcnt and expcnt not waited on
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// ---- wavefront reductions ----------------------------------------------------

// Sum over each row of sixteen lanes with DPP moves (no LDS traffic); every
// lane of the row gets a sum, lane 0 of the row always in the same order.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ float row16_sum(float v)
{
    v += dpp_mov<0x128>(v);   // row_ror:8
    v += dpp_mov<0x124>(v);   // row_ror:4
    v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    return v;
}

template <int WIDTH>
__device__ __forceinline__ float sum_lanes(float v)
{
#pragma unroll
    for (int o = WIDTH / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int WIDTH>
__device__ __forceinline__ double sum_lanes64(double v)
{
#pragma unroll
    for (int o = WIDTH / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace glrm
