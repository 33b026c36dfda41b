// range_mfma.hip — the range pass on the matrix cores.
//
// Sec. 3.2 writes the squared distance as |q|^2 + |x|^2 - 2 q.x with the
// norms precomputed, leaving the inner products as the dominant cost.  Here
// the inner products of a block of landmarks against all points form one
// dense contraction on v_mfma_f32_32x32x16_{bf16,f16}: landmarks are the M
// dimension (32 per panel, held in registers for the whole pass), points the
// N dimension (32 per tile, streamed from HBM in a swizzled layout so each
// 16-wide K step of a tile is one coalesced 1 KB load), accumulation in FP32
// starting from -RN32(|l|^2)/2.  The output G estimates (|x|^2 - D)/2.
//
// The epilogue is the delta-accurate oracle of Sec. 5.1 made exact: with the
// bound |G - (|x|^2 - D)/2| <= alpha |l|^2 + beta |x|^2 + abs (bounds.h), a
// pair is "out" when G <= U_x - alpha max|l|^2 and "in" when
// G > V_x + alpha max|l|^2 (max over the landmark panel); the rest — the band —
// is decided by the FP64 predicate (the verified range set of Sec. 5.3).
// With refine = 0 the pair is a member iff G > Z_x = (|x|^2 - e2)/2: a
// compressed-distance oracle with false negatives and false positives.
#include "dev_common.h"
#include "kernels.h"

namespace bm {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;
typedef __attribute__((ext_vector_type(16))) float f32x16;

// ---- operand preparation --------------------------------------------------------------

// float -> bf16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ double bf16_to_double(uint16_t h) { return (double)__uint_as_float((uint32_t)h << 16); }

template <int DT>
__global__ void k_mfma_operands(PointsView P, int kind, int S, uint16_t *Pop, uint16_t *Qop)
{
    const int64_t NT = (P.n + 31) / 32;
    const int64_t total = NT * S * 64;
    const int d = P.d;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(g & 63);
        const int64_t ts = g >> 6;
        const int s = (int)(ts % S);
        const int64_t t = ts / S;
        const int64_t p = t * 32 + (lane & 31);
        const int kb = 16 * s + 8 * (lane >> 5);
        uint16_t pv[8], qv[8];
        const int64_t row = p < P.n ? orig_index(P, p) * (int64_t)d : 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = kb + e;
            uint16_t a = 0, b = 0;
            if (p < P.n) {
                if (kind == MFMA_F16) {
                    if (k < d) a = b = ((const uint16_t *)P.X)[row + k];
                } else if (kind == MFMA_BF16) {
                    if (k < d) a = b = bf16_rne((float)load_coord<DT>(P.X, row + k));
                } else {   // three-product split: P = [hi|hi|lo], Q = [hi|lo|hi]
                    const int seg = k / d, kk = k - seg * d;
                    if (seg < 3) {
                        const double x = load_coord<DT>(P.X, row + kk);
                        const uint16_t hi = bf16_rne((float)x);
                        const uint16_t lo = bf16_rne((float)(x - bf16_to_double(hi)));
                        a = (seg == 2) ? lo : hi;
                        b = (seg == 1) ? lo : hi;
                    }
                }
            }
            pv[e] = a;
            qv[e] = b;
        }
        const int64_t o = g * 8;
        u32x4 wp, wq;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            wp[e] = (uint32_t)pv[2 * e] | ((uint32_t)pv[2 * e + 1] << 16);
            wq[e] = (uint32_t)qv[2 * e] | ((uint32_t)qv[2 * e + 1] << 16);
        }
        *(u32x4 *)(Pop + o) = wp;
        if (Qop != Pop) *(u32x4 *)(Qop + o) = wq;
    }
}

hipError_t launch_mfma_operands(const PointsView &P, int kind, int S, uint16_t *Pop, uint16_t *Qop, hipStream_t s)
{
    const int64_t total = ((P.n + 31) / 32) * S * 64;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 32768) blocks = 32768;
    if (P.dtype == 0) k_mfma_operands<0><<<(int)blocks, 256, 0, s>>>(P, kind, S, Pop, Qop);
    else if (P.dtype == 1) k_mfma_operands<1><<<(int)blocks, 256, 0, s>>>(P, kind, S, Pop, Qop);
    else k_mfma_operands<2><<<(int)blocks, 256, 0, s>>>(P, kind, S, Pop, Qop);
    return hipGetLastError();
}

// Neighbouring floats (subnormals are kept: the code is built without flushing).
__device__ __forceinline__ float next_up(float f)
{
    if (!(f < INFINITY)) return f;                       // +inf, NaN
    if (f == 0.0f) return __uint_as_float(1u);
    const uint32_t u = __float_as_uint(f);
    return __uint_as_float(f > 0.0f ? u + 1u : u - 1u);
}
__device__ __forceinline__ float next_down(float f) { return -next_up(-f); }

// Per-point scalars (rank order): the accumulator start, the rounded-up norm,
// and the three decision thresholds for this eps.  FP64 arithmetic, then a
// directed rounding to FP32 on the conservative side.
__device__ __forceinline__ float to_f32_down(double v)
{
    float f = (float)v;
    if ((double)f > v) f = next_down(f);
    return f;
}
__device__ __forceinline__ float to_f32_up(double v)
{
    float f = (float)v;
    if ((double)f < v) f = next_up(f);
    return f;
}

__global__ void k_mfma_scalars(int64_t n, const double *nu, MfmaBound b, double e2, double g64d, float *cinit,
                               float *nuup, float *U, float *V, float *Z)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double v = nu[r];
    const float nf = (float)v;
    cinit[r] = -0.5f * nf;
    nuup[r] = to_f32_up(v * (1.0 + g64d) * (1.0 + 1e-12));
    const double rel = 1e-12 * (v + b.t_out + 1.0);
    if (!b.sane) {
        U[r] = __builtin_nanf("");
        V[r] = __builtin_nanf("");
    } else {
        U[r] = to_f32_down((v - b.t_out) * 0.5 - b.beta * v - b.abs_err - rel);
        V[r] = to_f32_up((v - b.t_in) * 0.5 + b.beta * v + b.abs_err + rel);
    }
    Z[r] = (float)((v - e2) * 0.5);
}

hipError_t launch_mfma_scalars(int64_t n, const double *nu, const MfmaBound &b, double e2, int d, float *cinit,
                               float *nuup, float *U, float *V, float *Z, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const double g64d = (double)d * 0x1p-53 / (1.0 - (double)d * 0x1p-53);
    k_mfma_scalars<<<(int)((n + 255) / 256), 256, 0, s>>>(n, nu, b, e2, g64d, cinit, nuup, U, V, Z);
    return hipGetLastError();
}

// ---- the range pass ---------------------------------------------------------------------

template <bool F16>
__device__ __forceinline__ f32x16 mfma32(u32x4 a, u32x4 b, f32x16 c)
{
    if constexpr (F16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                      0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                       0, 0, 0);
}

// Row of the 32x32 output held in accumulator register i of this lane.
__device__ __forceinline__ int acc_row(int i, int half) { return 8 * (i >> 2) + 4 * half + (i & 3); }

constexpr int RM_THREADS = 256;

// One wave = MP panels of 32 landmarks x a contiguous range of 32-point tiles.
// KS = K steps per chunk (all of K when nch == 1).
template <int KS, int MP, bool F16>
__global__ __launch_bounds__(RM_THREADS) void k_range_mfma(MfmaArgs a, PointsView P, double e2,
                                                           const int32_t *__restrict__ A, const int64_t *blk,
                                                           RangeOut o, int NG, int64_t tpc, int nch)
{
    const int64_t ord0 = blk[0];
    const int na = (int)blk[1];
    const int lane = lane_id();
    const int col = lane & 31, half = lane >> 5;
    const int64_t wave = (int64_t)blockIdx.x * (RM_THREADS / 64) + (threadIdx.x >> 6);
    const int g = (int)(wave % NG);
    const int64_t c = wave / NG;
    const int pbase = g * MP;                       // first panel of this wave
    if (pbase * 32 >= na) return;                   // wave-uniform
    const int64_t NT = (P.n + 31) / 32;
    const int64_t t0 = c * tpc;
    const int64_t t1 = min(NT, t0 + tpc);
    if (t0 >= t1) return;
    const int S = a.S;

    // landmark ranks of this lane's A-operand rows and accumulator rows
    int32_t arank[MP];
    f32x16 cinit[MP];
    float aw[MP];
#pragma unroll
    for (int pi = 0; pi < MP; ++pi) {
        const int ai = (pbase + pi) * 32 + col;
        arank[pi] = ai < na ? A[ai] : -1;
        float nmax = ai < na ? a.nuup[arank[pi]] : 0.f;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nmax = fmaxf(nmax, __shfl_xor(nmax, off, 64));
        aw[pi] = next_up(a.alpha * nmax);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int aj = (pbase + pi) * 32 + acc_row(i, half);
            cinit[pi][i] = aj < na ? a.cinit[A[aj]] : 0.f;
        }
    }

    u32x4 areg[MP][KS];
    auto load_a = [&](int ch) {
#pragma unroll
        for (int pi = 0; pi < MP; ++pi)
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int ss = ch * KS + s;
                u32x4 v = {0u, 0u, 0u, 0u};
                if (arank[pi] >= 0 && ss < S) {
                    const int64_t r = arank[pi];
                    v = *(const u32x4 *)(a.Qop + ((((r >> 5) * S + ss) * 64) + (r & 31) + 32 * half) * 8);
                }
                areg[pi][s] = v;
            }
    };
    if (nch == 1) load_a(0);

    unsigned long long band = 0;
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t p = t * 32 + col;
        const bool pv = p < P.n;
        f32x16 acc[MP];
#pragma unroll
        for (int pi = 0; pi < MP; ++pi) acc[pi] = cinit[pi];
        for (int ch = 0; ch < nch; ++ch) {
            if (nch > 1) load_a(ch);
            u32x4 breg[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int ss = ch * KS + s;
                breg[s] = ss < S ? *(const u32x4 *)(a.Pop + (((t * S + ss) * 64) + lane) * 8)
                                 : u32x4{0u, 0u, 0u, 0u};
            }
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int pi = 0; pi < MP; ++pi) acc[pi] = mfma32<F16>(areg[pi][s], breg[s], acc[pi]);
        }

        bool cov = false;
        const float Ux = pv ? a.U[p] : INFINITY;
        const float Vx = pv ? a.V[p] : INFINITY;
        const float Zx = pv ? a.Z[p] : INFINITY;
        const int64_t xo = pv ? orig_index(P, p) : 0;
#pragma unroll
        for (int pi = 0; pi < MP; ++pi) {
            const int abase = (pbase + pi) * 32;
            if (abase >= na) break;                                      // wave-uniform
            uint32_t mem = 0;
            if (a.refine) {
                const float u = pv ? next_down(Ux - aw[pi]) : INFINITY;
                uint64_t any = 0;
#pragma unroll
                for (int i = 0; i < 16; ++i) any |= __ballot(!(acc[pi][i] <= u));
                if (!any) continue;                                      // every pair of the tile is out
                const float v = pv ? next_up(Vx + aw[pi]) : INFINITY;
                uint32_t bnd = 0;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const float gval = acc[pi][i];
                    const bool live = pv && (abase + acc_row(i, half) < na) && !(gval <= u);
                    if (live) {
                        if (gval > v) mem |= 1u << i;
                        else bnd |= 1u << i;
                    }
                }
                while (bnd) {
                    const int i = __builtin_ctz(bnd);
                    bnd &= bnd - 1;
                    ++band;
                    const int32_t lr = A[abase + acc_row(i, half)];
                    if (exact_member(P, orig_index(P, lr), xo, e2)) mem |= 1u << i;
                }
            } else {
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if (pv && abase + acc_row(i, half) < na && acc[pi][i] > Zx) mem |= 1u << i;
            }
            // append this lane's members with one atomic per wave
            const int cnt = __popc(mem);
            const uint64_t any_mem = __ballot(cnt != 0);
            if (!any_mem) continue;
            const int incl = wave_incl_scan(cnt);
            const int total = __shfl(incl, 63, 64);
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(&o.st->nkeys, (unsigned long long)total);
            base = __shfl(base, 0, 64) + (unsigned long long)(incl - cnt);
            cov |= cnt != 0;
            while (mem) {
                const int i = __builtin_ctz(mem);
                mem &= mem - 1;
                if (base < o.cap)
                    o.keys[base] = ((uint64_t)(ord0 + abase + acc_row(i, half)) << o.bn) | (uint64_t)xo;
                ++base;
            }
        }
        if (o.covered) {
            const uint64_t m = __ballot(cov);
            const uint64_t bits = (m | (m >> 32)) & 0xffffffffull;
            if (bits && lane == 0)
                atomicOr((unsigned long long *)&o.covered[(t * 32) >> 6], (unsigned long long)(bits << ((t * 32) & 63)));
        }
    }
    band = wave_sum(band);
    if (band && lane == 0) atomicAdd(&o.st->band, band);
}

// ---- self-check of the matrix-core behaviour the error bound relies on -------------------
// flags bit 0: bf16 32x32x16 output layout as acc_row() assumes; bit 1: same for f16;
// bit 2: f16 subnormal operands are multiplied exactly; bit 3: same for bf16.
__global__ void k_selfcheck(int *flags)
{
    const int lane = lane_id(), col = lane & 31, half = lane >> 5;
    // A = e_(m=5,k=11), B = e_(k=11,n=22): only D[5][22] = 1
    bf16x8 ab, bb;
    f16x8 ah, bh;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = 8 * half + e;
        const float va = (col == 5 && k == 11) ? 1.0f : 0.0f, vb = (col == 22 && k == 11) ? 1.0f : 0.0f;
        ab[e] = (__bf16)va;
        bb[e] = (__bf16)vb;
        ah[e] = (_Float16)va;
        bh[e] = (_Float16)vb;
    }
    const f32x16 z = {};
    const f32x16 db = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, bb, z, 0, 0, 0);
    const f32x16 dh = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, z, 0, 0, 0);
    bool okb = true, okh = true;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const float want = (acc_row(i, half) == 5 && col == 22) ? 1.0f : 0.0f;
        okb &= db[i] == want;
        okh &= dh[i] == want;
    }
    // subnormal operands in row 0 / column 0, k = 0
    f16x8 sa = {}, sb = {};
    bf16x8 ta = {}, tb = {};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        sa[e] = (_Float16)0.0f;
        sb[e] = (_Float16)0.0f;
        ta[e] = (__bf16)0.0f;
        tb[e] = (__bf16)0.0f;
    }
    if (lane == 0) {
        sa[0] = (_Float16)0x1p-20f;
        sb[0] = (_Float16)0x1p10f;
        ta[0] = (__bf16)0x1p-130f;
        tb[0] = (__bf16)0x1p100f;
    }
    const f32x16 ds = __builtin_amdgcn_mfma_f32_32x32x16_f16(sa, sb, z, 0, 0, 0);
    const f32x16 dt = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ta, tb, z, 0, 0, 0);
    const bool sub_h = ds[0] == 0x1p-10f, sub_b = dt[0] == 0x1p-30f;
    const uint64_t mb = __ballot(okb), mh = __ballot(okh);
    if (lane == 0)
        *flags = (mb == ~0ull ? 1 : 0) | (mh == ~0ull ? 2 : 0) | (sub_h ? 4 : 0) | (sub_b ? 8 : 0);
}

hipError_t run_selfcheck(int *flags_dev, hipStream_t s)
{
    k_selfcheck<<<1, 64, 0, s>>>(flags_dev);
    return hipGetLastError();
}

template <int KS, int MP, bool F16>
static hipError_t launch_ks(const MfmaArgs &a, const PointsView &P, double e2, const int32_t *A, const int64_t *blk,
                            int na_max, const RangeOut &o, int nch, hipStream_t s)
{
    const int npan = (na_max + 31) / 32;
    const int NG = (npan + MP - 1) / MP;
    const int64_t NT = (P.n + 31) / 32;
    // aim for about 8 waves per SIMD over the chip: 256 CUs x 4 SIMDs x 8
    const int64_t target_waves = 8192;
    int64_t chunks = (target_waves + NG - 1) / NG;
    if (chunks > NT) chunks = NT;
    if (chunks < 1) chunks = 1;
    const int64_t tpc = (NT + chunks - 1) / chunks;
    chunks = (NT + tpc - 1) / tpc;
    const int64_t waves = (int64_t)NG * chunks;
    const int64_t blocks = (waves + 3) / 4;
    k_range_mfma<KS, MP, F16><<<(unsigned)blocks, RM_THREADS, 0, s>>>(a, P, e2, A, blk, o, NG, tpc, nch);
    return hipGetLastError();
}

template <bool F16>
static hipError_t dispatch(const MfmaArgs &a, const PointsView &P, double e2, const int32_t *A, const int64_t *blk,
                           int na_max, const RangeOut &o, hipStream_t s)
{
    const int S = a.S;
    switch (S) {
    case 1: return launch_ks<1, 2, F16>(a, P, e2, A, blk, na_max, o, 1, s);
    case 2: return launch_ks<2, 2, F16>(a, P, e2, A, blk, na_max, o, 1, s);
    case 3: return launch_ks<3, 2, F16>(a, P, e2, A, blk, na_max, o, 1, s);
    case 4: return launch_ks<4, 2, F16>(a, P, e2, A, blk, na_max, o, 1, s);
    case 5: return launch_ks<5, 2, F16>(a, P, e2, A, blk, na_max, o, 1, s);
    case 6: return launch_ks<6, 2, F16>(a, P, e2, A, blk, na_max, o, 1, s);
    case 7: return launch_ks<7, 2, F16>(a, P, e2, A, blk, na_max, o, 1, s);
    case 8: return launch_ks<8, 2, F16>(a, P, e2, A, blk, na_max, o, 1, s);
    default: return launch_ks<8, 2, F16>(a, P, e2, A, blk, na_max, o, (S + 7) / 8, s);
    }
}

hipError_t launch_range_mfma(const MfmaArgs &a, const PointsView &P, double e2, const int32_t *A,
                             const int64_t *blk, int na_max, const RangeOut &o, hipStream_t s)
{
    if (P.n <= 0 || na_max <= 0) return hipSuccess;
    if (a.kind == MFMA_F16) return dispatch<true>(a, P, e2, A, blk, na_max, o, s);
    return dispatch<false>(a, P, e2, A, blk, na_max, o, s);
}

} // namespace bm
