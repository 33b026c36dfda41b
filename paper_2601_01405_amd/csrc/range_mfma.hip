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
#include <cstdlib>

#include "dev_common.h"
#include "kernels.h"

namespace bm {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
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
__global__ void k_mfma_operands(PointsView P, int kind, int S, double scale, uint16_t *Pop, uint16_t *Qop)
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
                    if (k < d) {
                        if constexpr (DT == 2) {
                            a = b = ((const uint16_t *)P.X)[row + k];          // stored float16: exact
                        } else {                                              // exact power-of-two scale,
                            const float v = (float)(load_coord<DT>(P.X, row + k) * scale);   // then RN to f16
                            a = b = __builtin_bit_cast(uint16_t, (_Float16)v);
                        }
                    }
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

hipError_t launch_mfma_operands(const PointsView &P, int kind, int S, double scale, uint16_t *Pop, uint16_t *Qop,
                                hipStream_t s)
{
    const int64_t total = ((P.n + 31) / 32) * S * 64;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 32768) blocks = 32768;
    if (P.dtype == 0) k_mfma_operands<0><<<(int)blocks, 256, 0, s>>>(P, kind, S, scale, Pop, Qop);
    else if (P.dtype == 1) k_mfma_operands<1><<<(int)blocks, 256, 0, s>>>(P, kind, S, scale, Pop, Qop);
    else k_mfma_operands<2><<<(int)blocks, 256, 0, s>>>(P, kind, S, scale, Pop, Qop);
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

__global__ void k_mfma_scalars(int64_t n, const double *nu, double nu_scale, MfmaBound b, double e2, double g64d,
                               float *cinit, float *nuup, float *U, float *V, float *Z)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double v = nu[r] * nu_scale;                 // working units (exact power-of-two scale)
    const float nf = (float)v;
    cinit[r] = -0.5f * nf;
    nuup[r] = to_f32_up(v * (1.0 + g64d) * (1.0 + 1e-12));
    const double rel = 1e-12 * (v + b.t_out + 1.0);
    if (!b.sane) {
        U[r] = __builtin_nanf("");
        V[r] = __builtin_nanf("");
    } else {
        // The kernel forms u = RN(U - w) and v = RN(V + w) with w >= alpha max|l|^2
        // widened by 2^-22; taking U and V 2^-23 further out keeps u <= U_exact - w_exact
        // and v >= V_exact + w_exact despite that rounding.
        const double u = (v - b.t_out) * 0.5 - b.beta * v - b.abs_err - rel;
        const double w = (v - b.t_in) * 0.5 + b.beta * v + b.abs_err + rel;
        U[r] = to_f32_down(u - 0x1p-23 * fabs(u) * (1.0 + 1e-9));
        V[r] = to_f32_up(w + 0x1p-23 * fabs(w) * (1.0 + 1e-9));
    }
    Z[r] = (float)((v - e2) * 0.5);
}

hipError_t launch_mfma_scalars(int64_t n, const double *nu, double nu_scale, const MfmaBound &b, double e2, int d,
                               float *cinit, float *nuup, float *U, float *V, float *Z, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const double g64d = (double)d * 0x1p-53 / (1.0 - (double)d * 0x1p-53);
    k_mfma_scalars<<<(int)((n + 255) / 256), 256, 0, s>>>(n, nu, nu_scale, b, e2, g64d, cinit, nuup, U, V, Z);
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

// Work split.  A workgroup of RM_WAVES waves owns RM_WAVES * RM_MP landmark
// panels of 32 (A operands and accumulator starts in registers for the whole
// pass) and a contiguous range of 32-point tiles.  Each tile's B operands and
// thresholds are staged once per workgroup in LDS (double buffered: the next
// tile's global loads are in flight while the current one is multiplied), so a
// point tile is read from memory once per RM_WAVES * RM_MP * 32 landmarks.
//
// MEMBERS mode appends (ordinal, point) keys and sets covered bits.  CONFLICT
// mode is the candidate-block resolve: landmarks and points are the same
// packed candidate set, and the output is C32[j * stride + p] = the bits r of
// rows i = 32 p + r < j whose ball holds candidate j, plus rowflag[j] = 1 when
// any bit is set.
constexpr int RM_WAVES = 8;
constexpr int RM_THREADS = RM_WAVES * 64;
constexpr int RM_MP = 2;

// Tiles per LDS stage: the next stage's loads have TPS tiles of matrix work
// to arrive in, and the workgroup synchronises once per stage.
#ifndef BM_STAGE_TILES
#define BM_STAGE_TILES 8
#endif
__host__ __device__ constexpr int stage_tiles(bool chunked, int ks)
{
    return chunked ? 1 : (ks <= 4 ? BM_STAGE_TILES : ks <= 6 ? (BM_STAGE_TILES + 1) / 2 : (BM_STAGE_TILES + 3) / 4);
}
// Staging vectors per thread for one stage: TPS tiles of S steps plus 96 thresholds each.
__host__ __device__ constexpr int stage_slots(int S, int tps) { return (tps * (S * 64 + 96) + RM_THREADS - 1) / RM_THREADS; }

// Point space of a MEMBERS pass: tiles [0, MT) are the settled list (entries
// < m valid), then rank tiles from rlo / 32 to the end.  A CONFLICT pass has
// no settled part.  The grid is NGW landmark groups x `chunks` point chunks
// (chunks a multiple of 8); the chunk length follows the device-side tile
// count.  Workgroups are dispatched to the 8 XCDs round robin, so the NGW
// groups of one chunk are placed on the same XCD and share its L2.
template <int KS, bool F16, bool CONFLICT, int SLOTS, bool CHUNKED>
__global__ __launch_bounds__(RM_THREADS) void k_range_mfma(MfmaArgs a, PointsView P, const int32_t *n_dev, double e2,
                                                           const int32_t *__restrict__ A, const int64_t *blk,
                                                           RangeOut o, SettledSet sd, uint32_t *C32, int c32_stride,
                                                           int *rowflag, int NGW, int chunks, int nch)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int S = a.S;
    // LDS: 2 buffers of TPS tiles of [S][64] u32x4 operands, then their thresholds
    constexpr int TPS = stage_tiles(CHUNKED, KS);
    const int buf_words = S * 64;                                  // u32x4 per tile
    u32x4 *sB = (u32x4 *)smem;                                     // [2][TPS][S*64]
    float *sT = (float *)(sB + 2 * TPS * buf_words);               // [2][TPS][3][32]
    float *sC = sT + 2 * TPS * 96;                                 // [RM_WAVES*RM_MP*32] accumulator starts
    float *sN = sC + RM_THREADS;                                   // [RM_WAVES*RM_MP*32] norm bounds

    const int64_t n = n_dev ? (int64_t)*n_dev : P.n;
    const int64_t ord0 = CONFLICT ? 0 : blk[0];
    const int na = CONFLICT ? (int)n : (int)blk[1];
    const int64_t msz = CONFLICT ? 0 : blk[3];                     // settled entries
    const int64_t MT = (msz + 31) / 32;                            // settled tiles
    const int64_t RT0 = CONFLICT ? 0 : (blk[2] >> 5);              // first rank tile
    const int wid = (int)(threadIdx.x >> 6), lane = lane_id(), col = lane & 31, half = lane >> 5;
    const int xcd = (int)(blockIdx.x & 7);
    const int kk = (int)(blockIdx.x >> 3);
    const int g = kk % NGW;
    const int64_t c = (int64_t)(kk / NGW) * 8 + xcd;
    if (g * RM_WAVES * RM_MP * 32 >= na) return;                   // workgroup-uniform
    const int64_t NT = (n + 31) / 32;
    const int64_t CT = MT + NT - RT0;                              // tiles of the point space
    const int64_t tpc = (CT + chunks - 1) / chunks;
    const int64_t t0 = c * tpc;
    const int64_t t1 = min(CT, t0 + tpc);
    if (t0 >= t1) return;                                          // workgroup-uniform
    const int pbase = (g * RM_WAVES + wid) * RM_MP;                // first panel of this wave
    const bool live = pbase * 32 < na;                             // wave-uniform

    // ---- the workgroup's landmarks: one per thread into LDS (start value, norm bound)
    static_assert(RM_WAVES * RM_MP * 32 == RM_THREADS, "one landmark per thread");
    {
        const int aj = g * RM_THREADS + (int)threadIdx.x;
        float cv = 0.f, nv = 0.f;
        if (aj < na) {
            const int32_t r = A ? A[aj] : aj;
            cv = a.cinit[r];
            nv = a.nuup[r];
        }
        sC[threadIdx.x] = cv;
        sN[threadIdx.x] = nv;
    }
    __syncthreads();

    // ---- this wave's panels: ranks, accumulator starts, norm bound, A operands
    int32_t arank[RM_MP];
    f32x16 cinit[RM_MP];
    float aw[RM_MP];
    u32x4 areg[RM_MP][KS];
#pragma unroll
    for (int pi = 0; pi < RM_MP; ++pi) {
        const int ai = (pbase + pi) * 32 + col;
        arank[pi] = ai < na ? (A ? A[ai] : ai) : -1;
        const int lbase = (wid * RM_MP + pi) * 32;                 // this panel in sC / sN
        float nmax = sN[lbase + col];
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) nmax = fmaxf(nmax, __shfl_xor(nmax, off, 64));
        const float w = next_up(a.alpha * nmax);
        aw[pi] = next_up(w + w * 0x1p-22f);          // see k_mfma_scalars: rounding slack
#pragma unroll
        for (int j = 0; j < 4; ++j) {                // rows 8j + 4 half + 0..3 of the panel
            const float4 q = *(const float4 *)(sC + lbase + 8 * j + 4 * half);
            cinit[pi][4 * j + 0] = q.x;
            cinit[pi][4 * j + 1] = q.y;
            cinit[pi][4 * j + 2] = q.z;
            cinit[pi][4 * j + 3] = q.w;
        }
    }
    auto load_a = [&](int ch) {
#pragma unroll
        for (int pi = 0; pi < RM_MP; ++pi)
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
    if (!CHUNKED && live) load_a(0);

    // ---- staging of one stage: TPS tiles x (S*64 operand vectors + 96 threshold floats)
    const int tile_items = buf_words + 96;
    const int items = TPS * tile_items;
    u32x4 pre[SLOTS];
    auto gload = [&](int64_t ts) {
#pragma unroll
        for (int k = 0; k < SLOTS; ++k) {
            const int it = (int)threadIdx.x + k * RM_THREADS;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (it < items) {
                const int tt = it / tile_items, r = it - tt * tile_items;
                const int64_t t = ts + tt;
                if (t < t1) {
                    const bool settled = t < MT;
                    const int64_t ts_ = settled ? t : RT0 + (t - MT);        // tile in its own array
                    if (r < buf_words) {
                        v = *(const u32x4 *)((settled ? sd.Pop : a.Pop) + ((ts_ * S) * 64 + r) * 8);
                    } else {
                        const int q = r - buf_words, which = q >> 5;
                        const int64_t pt = ts_ * 32 + (q & 31);
                        float f = INFINITY;
                        if (settled) f = which == 0 ? sd.U[pt] : which == 1 ? sd.V[pt] : sd.Z[pt];
                        else if (pt < n) f = which == 0 ? a.U[pt] : which == 1 ? a.V[pt] : a.Z[pt];
                        v[0] = __float_as_uint(f);
                    }
                }
            }
            pre[k] = v;
        }
    };
    // LDS per buffer: [TPS][S*64] operand vectors, then [TPS][96] thresholds
    auto lstore = [&](int buf) {
#pragma unroll
        for (int k = 0; k < SLOTS; ++k) {
            const int it = (int)threadIdx.x + k * RM_THREADS;
            if (it < items) {
                const int tt = it / tile_items, r = it - tt * tile_items;
                if (r < buf_words) sB[(buf * TPS + tt) * buf_words + r] = pre[k];
                else sT[(buf * TPS + tt) * 96 + (r - buf_words)] = __uint_as_float(pre[k][0]);
            }
        }
    };

    unsigned long long band = 0;
    // Let the setup loads (A operands, accumulator starts) land before the loop,
    // so the only loads in flight inside it are the next stage's staging loads
    // and the waitcnt pass need not wait for them before the matrix ops.
    __builtin_amdgcn_s_waitcnt(0);
    gload(t0);
    for (int64_t ts = t0; ts < t1; ts += TPS) {
        const int buf = (int)(((ts - t0) / TPS) & 1);
        lstore(buf);
        __syncthreads();
        if (ts + TPS < t1) gload(ts + TPS);
        if (!live) continue;
      for (int tt = 0; tt < TPS; ++tt) {
        const int64_t t = ts + tt;
        if (t >= t1) break;                                             // wave-uniform
        const int sb = (buf * TPS + tt) * buf_words;                    // this tile's operands in LDS
        const int stt = (buf * TPS + tt) * 96;                          // and thresholds
        const bool settled = t < MT;                                    // wave-uniform
        const int64_t tr = settled ? t : RT0 + (t - MT);                // tile in its own array
        const int64_t p = tr * 32 + col;                                // settled entry or rank
        const bool pv = settled ? p < msz : p < n;
        const float Ux = sT[stt + col], Vx = sT[stt + 32 + col], Zx = sT[stt + 64 + col];
        f32x16 acc[RM_MP];
        if (!CHUNKED) {
            u32x4 breg[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) breg[s] = sB[sb + s * 64 + lane];
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int pi = 0; pi < RM_MP; ++pi)
                    acc[pi] = mfma32<F16>(areg[pi][s], breg[s], s == 0 ? cinit[pi] : acc[pi]);
        } else {
#pragma unroll
            for (int pi = 0; pi < RM_MP; ++pi) acc[pi] = cinit[pi];
            for (int ch = 0; ch < nch; ++ch) {
                load_a(ch);
                u32x4 breg[KS];
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    const int ss = ch * KS + s;
                    breg[s] = ss < S ? sB[sb + ss * 64 + lane] : u32x4{0u, 0u, 0u, 0u};
                }
#pragma unroll
                for (int s = 0; s < KS; ++s)
#pragma unroll
                    for (int pi = 0; pi < RM_MP; ++pi) acc[pi] = mfma32<F16>(areg[pi][s], breg[s], acc[pi]);
            }
        }

        bool cov = false;
#pragma unroll
        for (int pi = 0; pi < RM_MP; ++pi) {
            const int abase = (pbase + pi) * 32;
            if (abase >= na) break;                                      // wave-uniform
            const f32x16 av = acc[pi];
            // u, v: conservative thresholds for this point and panel (U, V and aw carry
            // the slack for these two roundings); +inf for padding points
            const float u = Ux - aw[pi];
            if (!CONFLICT) {
                // fast path: is any pair of the 32x32 tile possibly a member?
                const float cut = a.refine ? u : Zx;
                float m = fmaxf(fmaxf(av[0], av[1]), av[2]);
                m = fmaxf(fmaxf(m, av[3]), av[4]);
                m = fmaxf(fmaxf(m, av[5]), av[6]);
                m = fmaxf(fmaxf(m, av[7]), av[8]);
                m = fmaxf(fmaxf(m, av[9]), av[10]);
                m = fmaxf(fmaxf(m, av[11]), av[12]);
                m = fmaxf(fmaxf(m, av[13]), av[14]);
                m = fmaxf(m, av[15]);
                if (!__ballot(!(m <= cut))) continue;
            }
            uint32_t mem = 0;
            const int64_t xo = !pv ? 0 : settled ? (int64_t)sd.idx[p] : orig_index(P, p);
            if (a.refine) {
                const float v = Vx + aw[pi];
                uint32_t bnd = 0;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const float gval = av[i];
                    const int ai = abase + acc_row(i, half);
                    bool ok = pv && ai < na && !(gval <= u);
                    if (CONFLICT) ok = ok && ai < p;
                    if (ok) {
                        if (gval > v) mem |= 1u << i;
                        else bnd |= 1u << i;
                    }
                }
                while (bnd) {
                    const int i = __builtin_ctz(bnd);
                    bnd &= bnd - 1;
                    ++band;
                    const int ai = abase + acc_row(i, half);
                    const int32_t lr = A ? A[ai] : ai;
                    if (exact_member(P, orig_index(P, lr), xo, e2)) mem |= 1u << i;
                }
            } else {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int ai = abase + acc_row(i, half);
                    if (pv && ai < na && (!CONFLICT || ai < p) && av[i] > Zx) mem |= 1u << i;
                }
            }
            if (CONFLICT) {
                uint32_t w = 0;
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if ((mem >> i) & 1u) w |= 1u << acc_row(i, half);
                w |= __shfl_xor(w, 32, 64);
                if (half == 0 && pv) {
                    C32[p * c32_stride + (pbase + pi)] = w;
                    if (w) rowflag[p] = 1;
                }
                continue;
            }
            // append this lane's members with one atomic per wave
            const int cnt = __popc(mem);
            if (!__ballot(cnt != 0)) continue;
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
        if (!CONFLICT && o.covered && !settled) {
            const uint64_t m = __ballot(cov);
            const uint64_t bits = (m | (m >> 32)) & 0xffffffffull;
            if (bits && lane == 0)
                atomicOr((unsigned long long *)&o.covered[(tr * 32) >> 6], (unsigned long long)(bits << ((tr * 32) & 63)));
        }
      }
    }
    band = wave_sum(band);
    if (band && lane == 0 && o.st) atomicAdd(&o.st->band, band);
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

template <int KS, bool F16, bool CONFLICT, int SLOTS, bool CHUNKED>
static hipError_t launch_ks(const MfmaArgs &a, const PointsView &P, const int32_t *n_dev, double e2, const int32_t *A,
                            const int64_t *blk, int na_max, int64_t n_max, const RangeOut &o, const SettledSet &sd,
                            uint32_t *C32, int c32_stride, int *rowflag, int nch, hipStream_t s)
{
    const int npan = (na_max + 31) / 32;
    const int per_wg = RM_WAVES * RM_MP;
    const int NGW = (npan + per_wg - 1) / per_wg;
    const int64_t NT = (n_max + 31) / 32 + 1;                      // + a partial settled tile
    // about one workgroup per CU (256 CUs) unless BM_RANGE_WORKGROUPS says otherwise
    static const int64_t env_wg = [] {
        const char *e = getenv("BM_RANGE_WORKGROUPS");
        return e ? atoll(e) : 0LL;
    }();
    const int64_t target_wg = env_wg > 0 ? env_wg : 256;
    int64_t chunks = (target_wg + NGW - 1) / NGW;
    if (chunks > NT) chunks = NT;
    chunks = (chunks + 7) / 8 * 8;                                  // whole XCD rounds
    const int64_t wgs = (int64_t)NGW * chunks;
    constexpr int TPS = stage_tiles(CHUNKED, KS);
    const size_t shmem = (size_t)2 * TPS * (a.S * 64 * 16 + 96 * sizeof(float)) + 2 * RM_THREADS * sizeof(float);
    k_range_mfma<KS, F16, CONFLICT, SLOTS, CHUNKED><<<(unsigned)wgs, RM_THREADS, shmem, s>>>(
        a, P, n_dev, e2, A, blk, o, sd, C32, c32_stride, rowflag, NGW, (int)chunks, nch);
    return hipGetLastError();
}

template <bool F16, bool CONFLICT>
static hipError_t dispatch(const MfmaArgs &a, const PointsView &P, const int32_t *n_dev, double e2, const int32_t *A,
                           const int64_t *blk, int na_max, int64_t n_max, const RangeOut &o, const SettledSet &sd,
                           uint32_t *C32, int c32_stride, int *rowflag, hipStream_t s)
{
#define BM_KS(k, nch, slots) \
    launch_ks<k, F16, CONFLICT, slots, (nch > 1)>(a, P, n_dev, e2, A, blk, na_max, n_max, o, sd, C32, c32_stride, rowflag, \
                                                  nch, s)
    switch (a.S) {
    case 1: return BM_KS(1, 1, stage_slots(1, stage_tiles(false, 1)));
    case 2: return BM_KS(2, 1, stage_slots(2, stage_tiles(false, 2)));
    case 3: return BM_KS(3, 1, stage_slots(3, stage_tiles(false, 3)));
    case 4: return BM_KS(4, 1, stage_slots(4, stage_tiles(false, 4)));
    case 5: return BM_KS(5, 1, stage_slots(5, stage_tiles(false, 5)));
    case 6: return BM_KS(6, 1, stage_slots(6, stage_tiles(false, 6)));
    case 7: return BM_KS(7, 1, stage_slots(7, stage_tiles(false, 7)));
    case 8: return BM_KS(8, 1, stage_slots(8, stage_tiles(false, 8)));
    default: return launch_ks<8, F16, CONFLICT, stage_slots(kMaxMfmaSteps, stage_tiles(true, 8)), true>(
                 a, P, n_dev, e2, A, blk, na_max, n_max, o, sd, C32, c32_stride, rowflag, (a.S + 7) / 8, s);
    }
#undef BM_KS
}

hipError_t launch_range_mfma(const MfmaArgs &a, const PointsView &P, double e2, const int32_t *A,
                             const int64_t *blk, int na_max, const RangeOut &o, const SettledSet &sd, hipStream_t s)
{
    if (a.S > kMaxMfmaSteps) return hipErrorInvalidValue;
    if (P.n <= 0 || na_max <= 0) return hipSuccess;
    if (a.kind == MFMA_F16)
        return dispatch<true, false>(a, P, nullptr, e2, A, blk, na_max, P.n, o, sd, nullptr, 0, nullptr, s);
    return dispatch<false, false>(a, P, nullptr, e2, A, blk, na_max, P.n, o, sd, nullptr, 0, nullptr, s);
}

hipError_t launch_resolve_mfma(const MfmaArgs &packed, const PointsView &Pc, const int32_t *nc_dev, double e2, int B,
                               uint32_t *C32, int *rowflag, GreedyState *st, hipStream_t s)
{
    if (packed.S > kMaxMfmaSteps) return hipErrorInvalidValue;
    RangeOut o{nullptr, nullptr, 0, st, 0};
    const SettledSet none{};
    const int stride = 2 * ((B + 63) / 64);
    if (packed.kind == MFMA_F16)
        return dispatch<true, true>(packed, Pc, nc_dev, e2, nullptr, nullptr, B, B, o, none, C32, stride, rowflag, s);
    return dispatch<false, true>(packed, Pc, nc_dev, e2, nullptr, nullptr, B, B, o, none, C32, stride, rowflag, s);
}

// Copy the gathered candidates' operands and scalars into a packed set
// (candidate j in place of rank j) for the resolve, and their original indices.
__global__ void k_pack_candidates(MfmaArgs a, const int32_t *cand, const GreedyState *st, const int32_t *perm, int B,
                                  MfmaArgs out, int32_t *cand_orig)
{
    const int nc = st->nc;
    const int S = a.S;
    const int64_t Bp = ((B + 31) / 32) * 32;
    const int64_t nvec = Bp * S * 2;                 // (candidate, step, half) 16-byte vectors
    const bool two = a.Qop != a.Pop;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < nvec + Bp;
         g += (int64_t)gridDim.x * blockDim.x) {
        if (g < nvec) {
            const int half = (int)(g & 1);
            const int64_t js = g >> 1;
            const int st_ = (int)(js % S);
            const int64_t j = js / S;
            const int64_t dst = ((((j >> 5) * S + st_) * 64) + (j & 31) + 32 * half) * 8;
            u32x4 vp = {0u, 0u, 0u, 0u}, vq = {0u, 0u, 0u, 0u};
            if (j < nc) {
                const int64_t r = cand[j];
                const int64_t src = ((((r >> 5) * S + st_) * 64) + (r & 31) + 32 * half) * 8;
                vp = *(const u32x4 *)(a.Pop + src);
                if (two) vq = *(const u32x4 *)(a.Qop + src);
            }
            *(u32x4 *)((uint16_t *)out.Pop + dst) = vp;
            if (two) *(u32x4 *)((uint16_t *)out.Qop + dst) = vq;
        } else {
            const int64_t j = g - nvec;
            const bool v = j < nc;
            const int32_t r = v ? cand[j] : 0;
            ((float *)out.cinit)[j] = v ? a.cinit[r] : 0.f;
            ((float *)out.nuup)[j] = v ? a.nuup[r] : 0.f;
            ((float *)out.U)[j] = v ? a.U[r] : INFINITY;
            ((float *)out.V)[j] = v ? a.V[r] : INFINITY;
            ((float *)out.Z)[j] = v ? a.Z[r] : INFINITY;
            cand_orig[j] = v ? (perm ? perm[r] : r) : 0;
        }
    }
}

hipError_t launch_pack_candidates(const MfmaArgs &a, const int32_t *cand, const GreedyState *st, const int32_t *perm,
                                  int B, const MfmaArgs &out, int32_t *cand_orig, hipStream_t s)
{
    const int64_t Bp = ((B + 31) / 32) * 32;
    const int64_t total = Bp * a.S * 2 + Bp;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_pack_candidates<<<(int)blocks, 256, 0, s>>>(a, cand, st, perm, B, out, cand_orig);
    return hipGetLastError();
}

} // namespace bm
