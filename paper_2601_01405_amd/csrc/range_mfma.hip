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
#include <algorithm>
#include <cstdlib>

#include <hip/hip_ext.h>

#include "dev_common.h"
#include "greedy_dev.h"
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
        // float32 rows of a multiple of 8 coordinates on a 16-byte aligned array:
        // the thread's 8 coordinates (one segment of the split) are read as two
        // float4 loads; the values, and so the operands, are the same
        float xv[8] = {};
        const bool vec = DT == 1 && (d & 7) == 0 && ((uintptr_t)P.X & 15u) == 0;   // uniform
        if (vec && p < P.n) {
            const int kk0 = kind == MFMA_F16 || kind == MFMA_BF16 ? kb : kb - (kb / d) * d;
            if ((kind == MFMA_F16 || kind == MFMA_BF16) ? kb < d : kb / d < 3) {
                const BM_GLOBAL u32x4 *src = (const BM_GLOBAL u32x4 *)((const BM_GLOBAL float *)P.X + row + kk0);
                const u32x4 u0 = src[0], u1 = src[1];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    xv[e] = __uint_as_float(u0[e]);
                    xv[4 + e] = __uint_as_float(u1[e]);
                }
            }
        }
        auto coord = [&](int e, int64_t off) -> double {
            if constexpr (DT == 1) {
                if (vec) return (double)xv[e];
            }
            return load_coord<DT>(P.X, off);
        };
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
                            const float v = (float)(coord(e, row + k) * scale);   // then RN to f16
                            a = b = __builtin_bit_cast(uint16_t, (_Float16)v);
                        }
                    }
                } else if (kind == MFMA_BF16) {
                    if (k < d) a = b = bf16_rne((float)coord(e, row + k));
                } else {   // three-product split: P = [hi|hi|lo], Q = [hi|lo|hi]
                    const int seg = k / d, kk = k - seg * d;
                    if (seg < 3) {
                        const double x = coord(e, row + kk);
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
                               float *cinit, float *nuup, float *T3)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t np = (n + 31) / 32 * 32;
    if (r >= np) return;
    if (r >= n) {                                      // padding of the last tile: never a member
        T3[t3_index(r, T3_U)] = INFINITY;
        T3[t3_index(r, T3_V)] = INFINITY;
        T3[t3_index(r, T3_Z)] = INFINITY;
        return;
    }
    const double v = nu[r] * nu_scale;                 // working units (exact power-of-two scale)
    const float nf = (float)v;
    cinit[r] = -0.5f * nf;
    nuup[r] = to_f32_up(v * (1.0 + g64d) * (1.0 + 1e-12));
    const double rel = 1e-12 * (v + b.t_out + 1.0);
    float U, V;
    if (!b.sane) {
        U = __builtin_nanf("");
        V = __builtin_nanf("");
    } else {
        // The kernel forms u = RN(U - w) and v = RN(V + w) with w >= alpha max|l|^2
        // widened by 2^-22; taking U and V 2^-23 further out keeps u <= U_exact - w_exact
        // and v >= V_exact + w_exact despite that rounding.
        const double u = (v - b.t_out) * 0.5 - b.beta * v - b.abs_err - rel;
        const double w = (v - b.t_in) * 0.5 + b.beta * v + b.abs_err + rel;
        U = to_f32_down(u - 0x1p-23 * fabs(u) * (1.0 + 1e-9));
        V = to_f32_up(w + 0x1p-23 * fabs(w) * (1.0 + 1e-9));
    }
    T3[t3_index(r, T3_U)] = U;
    T3[t3_index(r, T3_V)] = V;
    T3[t3_index(r, T3_Z)] = (float)((v - e2) * 0.5);
}

hipError_t launch_mfma_scalars(int64_t n, const double *nu, double nu_scale, const MfmaBound &b, double e2, int d,
                               float *cinit, float *nuup, float *T3, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t np = (n + 31) / 32 * 32;
    const double g64d = (double)d * 0x1p-53 / (1.0 - (double)d * 0x1p-53);
    k_mfma_scalars<<<(int)((np + 255) / 256), 256, 0, s>>>(n, nu, nu_scale, b, e2, g64d, cinit, nuup, T3);
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
// pass) and a contiguous range of 32-point tiles.  Tiles are staged through
// LDS in stages of TPS tiles, double buffered, with two register sets of
// staging loads: while stage s is multiplied, the loads of stages s+1 and s+2
// are in flight, so memory latency has two stage-times to hide behind.  A
// point tile is read from memory once per RM_WAVES * RM_MP * 32 landmarks.
//
// MEMBERS mode appends (ordinal, point) keys and sets covered bits.  CONFLICT
// mode is the candidate-block resolve: landmarks and points are both the
// block's candidates (rank A[j] for candidate j, read in place), and the
// output is C32[j * stride + p] = the bits r of rows i = 32 p + r < j whose
// ball holds candidate j, for the panels p with 32 p < j, plus rowflag[j] = 1
// when any bit is set.  The words start at zero and only nonzero ones are
// stored (the accept clears the rows it read), so a pass over a block with
// few conflicts writes almost nothing.  Tiles that lie wholly above the
// diagonal are skipped.
//
// Point space of a MEMBERS pass: tiles [0, MT) are the settled list (entries
// < m valid), then rank tiles from rlo / 32 to the end.  A CONFLICT pass has
// no settled part.  The grid is NGW landmark groups x `chunks` point chunks
// (chunks a multiple of 8); the chunk length follows the device-side tile
// count.  Workgroups are dispatched to the 8 XCDs round robin, so the NGW
// groups of one chunk are placed on the same XCD and share its L2.
constexpr int RM_WAVES = 8;
constexpr int RM_THREADS = RM_WAVES * 64;
constexpr int RM_MP = 2;

// Tiles per LDS stage (16-55 KB of operands per stage); one tile when the
// K steps are processed in chunks of 8.  From K = 48 (three steps) on, except
// at four steps where the LDS does not allow it, a stage holds twice the tiles
// of the two-register-set scheme and is staged through one register set: the
// next stage's loads have a whole (long) stage to arrive, and the workgroup
// meets at half as many barriers.
__host__ __device__ constexpr int stage_tiles_two_sets(int ks)
{
    return ks <= 2 ? 16 : ks <= 4 ? 8 : ks <= 6 ? 4 : 2;
}
__host__ __device__ constexpr bool one_set(bool chunked, int ks) { return !chunked && ks >= 3 && ks != 4; }
__host__ __device__ constexpr int stage_tiles(bool chunked, int ks)
{
    return chunked ? 1 : one_set(chunked, ks) ? 2 * stage_tiles_two_sets(ks) : stage_tiles_two_sets(ks);
}
// Operand vectors of one stage, and per thread.
__host__ __device__ constexpr int stage_vecs(bool chunked, int ks)
{
    return stage_tiles(chunked, ks) * (chunked ? kMaxMfmaSteps : ks) * 64;
}
__host__ __device__ constexpr int op_slots(bool chunked, int ks)
{
    return (stage_vecs(chunked, ks) + RM_THREADS - 1) / RM_THREADS;
}

// Workgroup exit: the execution-clock window, then, for a task with a chain
// step, a ticket; the task's last workgroup to finish runs the chain's next
// serial step (accept after a resolve, open the next block after a range
// pass).  No workgroup waits for another.
template <bool CONFLICT>
__device__ void range_wg_exit(const RangeTask &T, KernelClock *clk, unsigned char *smem)
{
    __syncthreads();                                               // every wave's stores have reached L2
    clock_leave(clk);
    const ChainTask *chain = T.chain;
    if (!chain) return;                                            // workgroup-uniform
    __shared__ int sh_last;
    if (threadIdx.x == 0) {
        GreedyState *st = chain->st;
        // One agent-scope release per workgroup (it writes back this XCD's L2,
        // which holds the whole workgroup's stores), one acquire in the last.
        const unsigned int tk = __hip_atomic_fetch_add(&st->ticket, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const bool last = tk + 1u == (unsigned int)T.NGW * (unsigned int)T.chunks;
        if (last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");     // every workgroup's writes are visible
            st->ticket = 0u;                                       // for the chain's next launch
        }
        sh_last = last ? 1 : 0;
    }
    __syncthreads();                                               // (the acquire invalidated the CU's caches)
    if (!sh_last) return;
    const unsigned long long t_in = clk ? (unsigned long long)wall_clock64() : 0ull;
    if (CONFLICT) block_accept<RM_THREADS>(*chain, smem);
    else block_open<RM_THREADS>(*chain, smem);
    if (clk) {
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(&clk->tail, (unsigned long long)wall_clock64() - t_in);
    }
}

// LDS of a range workgroup: the double-buffered stages, the accumulator
// starts and norm bounds, one band queue per wave (queue_cap entries), and a
// key stage: members are appended there with LDS atomics and written out in
// chunks at stage barriers, one global atomic per chunk, so that the key
// counter (one per build, or per batch) is not hit once per wave and panel.
constexpr int kKeyStage = 2048;
constexpr size_t kLdsBudget = 160 * 1024;                          // LDS of one workgroup on gfx950
__host__ __device__ constexpr size_t queue_offset(int S, int TPS)
{
    return (size_t)2 * TPS * (S * 64 * 16 + 24 * 16) + 2 * RM_THREADS * sizeof(float);
}
// Band-queue entries per wave: what the stages and the key stage leave of the
// budget (1 KB kept for the kernel's own variables), 64 to 1024, a multiple of 64.
__host__ __device__ constexpr int queue_cap(int S, int TPS)
{
    const size_t used = queue_offset(S, TPS) + (size_t)kKeyStage * 8 + 16 + 1024;
    const size_t q = used < kLdsBudget ? (kLdsBudget - used) / ((size_t)RM_WAVES * 8) : 0;
    const size_t c = q > 1024 ? 1024 : q;
    return (int)(c < 64 ? 64 : (c / 64) * 64);
}
__host__ __device__ constexpr size_t key_stage_offset(int S, int TPS)
{
    return queue_offset(S, TPS) + (size_t)RM_WAVES * queue_cap(S, TPS) * 8;
}
__host__ __device__ constexpr size_t range_lds_bytes(int S, int TPS)
{
    return key_stage_offset(S, TPS) + (size_t)kKeyStage * 8 + 16;
}

template <int KS, bool F16, bool CONFLICT, bool CHUNKED>
__global__ __launch_bounds__(RM_THREADS) void k_range_mfma(const RangeTask *__restrict__ tasks,
                                                           const int32_t *__restrict__ task_of, int nch,
                                                           KernelClock *clk)
{
    clock_enter(clk);
    constexpr int TPS = stage_tiles(CHUNKED, KS);
    constexpr int OPS = op_slots(CHUNKED, KS);
    constexpr int THV = TPS * 24;                                  // threshold vectors per stage
    static_assert(THV <= RM_THREADS, "one threshold vector per thread");
    extern __shared__ __align__(16) unsigned char smem[];
    const RangeTask &T = tasks[task_of ? task_of[blockIdx.x] : 0];
    const MfmaArgs a = T.a;
    const PointsView P = T.P;
    const double e2 = T.e2;
    const BM_GLOBAL int32_t *A = gbl(T.A);
    const RangeOut o = T.o;
    const SettledSet sd = T.sd;
    const int S = CHUNKED ? a.S : KS;
    const int tile_vecs = S * 64;                                  // operand vectors of one tile
    const int buf_vecs = TPS * tile_vecs;
    u32x4 *sB = (u32x4 *)smem;                                     // [2][TPS][S*64] operands
    u32x4 *sT = sB + 2 * buf_vecs;                                 // [2][TPS][24]: U[32] V[32] Z[32]
    float *sC = (float *)(sT + 2 * THV);                           // [RM_THREADS] accumulator starts
    float *sN = sC + RM_THREADS;                                   // [RM_THREADS] norm bounds

    const int64_t n = T.n_dev ? (int64_t)*gbl(T.n_dev) : P.n;
    const BM_GLOBAL int64_t *blk = gbl(T.blk);
    const int64_t ord0 = CONFLICT ? 0 : blk[0];
    const int na = CONFLICT ? (int)n : (int)blk[1];
    const int64_t msz = CONFLICT ? 0 : blk[3];                     // settled entries
    const int MT = (int)((msz + 31) / 32);                         // settled tiles
    const int RT0 = CONFLICT ? 0 : (int)(blk[2] >> 5);             // first rank tile
    const int tid = (int)threadIdx.x;
    const int wid = tid >> 6, lane = lane_id(), col = lane & 31, half = lane >> 5;
    const int lb = (int)blockIdx.x - T.wg0;                        // workgroup within the task
    // The launch is sized for a full block; its workgroups are spread over the
    // landmark groups this pass actually has (fewer once candidates are
    // rejected or a chain ends), in whole rounds of 8 (one per XCD).
    const int launched = T.NGW * T.chunks;
    // a resolve first copies its share of the entries the opening settled
    // (the range pass after it reads them)
    if (CONFLICT && T.chain) settle_copy<RM_THREADS>(*T.chain, lb, launched);
    // Workgroup -> (landmark group g, tiles [t0, t1)).  A range pass: the
    // workgroups go to ceil(na / 512) groups times `chunks` point chunks, the
    // groups of one chunk on one XCD.  A resolve needs, for group g, only the
    // tiles from 16 g on (candidates past the group's first row): that
    // triangle is cut into pieces of `per` tiles, so that its longest
    // workgroup does about the mean work.
    int g, c = -1, t0, t1;
    const int NT = (int)((n + 31) / 32);
    if constexpr (CONFLICT) {
        const int ngw = max(1, (na + RM_THREADS - 1) / RM_THREADS);
        int work = 0;
        for (int gg = 0; gg < ngw; ++gg) work += max(0, NT - 16 * gg);
        const int slots = max(1, launched - ngw);
        const int per = max(1, (work + slots - 1) / slots);
        g = -1;
        t0 = t1 = 0;
        for (int gg = 0, acc = 0; gg < ngw; ++gg) {
            const int len = max(0, NT - 16 * gg);
            const int kg = (len + per - 1) / per;
            if (lb < acc + kg) {
                g = gg;
                t0 = 16 * gg + (lb - acc) * per;
                t1 = min(NT, t0 + per);
                break;
            }
            acc += kg;
        }
        if (g < 0 || g * RM_THREADS >= na || t0 >= t1) {           // workgroup-uniform
            range_wg_exit<CONFLICT>(T, clk, smem);
            return;
        }
    } else {
        const int NGW = max(1, min((na + RM_THREADS - 1) / RM_THREADS, launched / 8));
        const int chunks = launched / NGW / 8 * 8;
        if (lb >= NGW * chunks) {                                  // workgroup-uniform
            range_wg_exit<CONFLICT>(T, clk, smem);
            return;
        }
        const int xcd = lb & 7;
        const int kk = lb >> 3;
        g = kk % NGW;
        c = (kk / NGW) * 8 + xcd;
        // the landmark bits of this pass's landmarks (one workgroup per landmark
        // group sets them; the next block's settle step reads them after the pass)
        if (c == 0 && T.chain && T.chain->settle) {
            const int aj = g * RM_THREADS + tid;
            if (aj < na) {
                const int32_t r = A ? A[aj] : aj;
                gatomic_or((unsigned long long *)&T.chain->islm[r >> 6], 1ull << (r & 63));
            }
        }
        if (g * RM_WAVES * RM_MP * 32 >= na) {                     // workgroup-uniform
            range_wg_exit<CONFLICT>(T, clk, smem);
            return;
        }
        const int CT = MT + NT - RT0;                              // tiles of the point space
        const int tpc = (CT + chunks - 1) / chunks;
        t0 = c * tpc;
        t1 = min(CT, t0 + tpc);
        if (t0 >= t1) {                                            // workgroup-uniform
            range_wg_exit<CONFLICT>(T, clk, smem);
            return;
        }
    }
    const int pbase = (g * RM_WAVES + wid) * RM_MP;                // first panel of this wave
    const bool live = pbase * 32 < na;                             // wave-uniform

    // ---- the workgroup's landmarks: one per thread into LDS (start value, norm bound)
    static_assert(RM_WAVES * RM_MP * 32 == RM_THREADS, "one landmark per thread");
    {
        const int aj = g * RM_THREADS + tid;
        float cv = 0.f, nv = 0.f;
        if (aj < na) {
            const int32_t r = A ? A[aj] : aj;
            cv = gbl(a.cinit)[r];
            nv = gbl(a.nuup)[r];
        }
        sC[tid] = cv;
        sN[tid] = nv;
    }
    uint64_t *kst = (uint64_t *)(smem + key_stage_offset(CHUNKED ? a.S : KS, TPS));
    int *kst_n = (int *)(kst + kKeyStage);
    // kst_seen[s & 1]: the stage count as thread 0 saw it early in stage s.  A
    // flush in stage s is decided on kst_seen[(s - 1) & 1], which no one writes
    // during stage s, so every wave takes the same decision.
    __shared__ int kst_seen[2];
    __shared__ unsigned long long sh_kbase;
    if (!CONFLICT && tid == 0) {
        *kst_n = 0;
        kst_seen[0] = kst_seen[1] = 0;
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
                    v = *(const BM_GLOBAL u32x4 *)gbl(a.Qop + ((((r >> 5) * S + ss) * 64) + (r & 31) + 32 * half) * 8);
                }
                areg[pi][s] = v;
            }
    };
    if (!CHUNKED && live) load_a(0);

    // ---- staging.  Slot k of this thread always carries operand vector
    // tid + k * RM_THREADS of a stage (tile op_tt[k], vector op_rem[k] of it),
    // and thread tid < THV one threshold vector (tile th_tt, floats 4 th_q ..).
    int op_tt[OPS], op_rem[OPS];
#pragma unroll
    for (int k = 0; k < OPS; ++k) {
        const int it = tid + k * RM_THREADS;
        op_tt[k] = it < buf_vecs ? it / tile_vecs : -1;
        op_rem[k] = it - (it / tile_vecs) * tile_vecs;
    }
    const int th_tt = tid < THV ? tid / 24 : -1;
    const int th_q = tid - (tid / 24) * 24;
    u32x4 preA[OPS], preB[OPS];
    u32x4 pretA, pretB;
    // tile t of the point space -> its own array and the tile index in it
    // Every load is issued (tiles past t1 and unused slots read tile t0 again,
    // in bounds, and are never consumed), so the number of loads per stage is
    // fixed and the waits before a store can leave the younger stage in flight.
    // A resolve reads its candidates in place: candidate j is rank A[j] (slots
    // past the count repeat the last candidate and are masked out later).
    auto gload = [&](int ts, u32x4 (&pre)[OPS], u32x4 &pre_t) {
#pragma unroll
        for (int k = 0; k < OPS; ++k) {
            int t = ts + op_tt[k];
            t = (op_tt[k] >= 0 && t < t1) ? t : t0;
            const int rem = op_tt[k] >= 0 ? op_rem[k] : 0;
            if (CONFLICT) {
                const int sl = rem >> 6, ln = rem & 63;                 // step and lane of the vector
                const int64_t r = A[min((int64_t)t * 32 + (ln & 31), n - 1)];
                pre[k] = *(const BM_GLOBAL u32x4 *)gbl(a.Pop + ((((r >> 5) * S + sl) * 64) + (r & 31) + 32 * (ln >> 5)) * 8);
            } else {
                const bool stl = t < MT;
                const int64_t tl = stl ? t : t - MT + RT0;
                const uint16_t *base = stl ? sd.Pop : a.Pop;
                pre[k] = *(const BM_GLOBAL u32x4 *)gbl(base + (tl * tile_vecs + rem) * 8);
            }
        }
        {
            int t = ts + th_tt;
            t = (th_tt >= 0 && t < t1) ? t : t0;
            const int q = th_tt >= 0 ? th_q : 0;
            if (CONFLICT) {                                             // U, V or Z of four candidates
                const int which = q >> 3, p0 = 4 * (q & 7);
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    v[e] = gbl(a.T3)[t3_index(A[min((int64_t)t * 32 + p0 + e, n - 1)], which)];
                pre_t = u32x4{__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                              __float_as_uint(v[3])};
            } else {
                const bool stl = t < MT;
                const int64_t tl = stl ? t : t - MT + RT0;
                const float *base = stl ? sd.T3 : a.T3;
                pre_t = *(const BM_GLOBAL u32x4 *)gbl(base + tl * 96 + q * 4);
            }
        }
    };
    auto lstore = [&](int buf, const u32x4 (&pre)[OPS], const u32x4 &pre_t) {
#pragma unroll
        for (int k = 0; k < OPS; ++k)
            if (op_tt[k] >= 0) sB[buf * buf_vecs + tid + k * RM_THREADS] = pre[k];
        if (th_tt >= 0) sT[buf * THV + tid] = pre_t;
    };

    unsigned long long band = 0;
    const int thr_off = a.refine ? 0 : 64;                         // screen on U (refined) or Z

    // Band queue of this wave (refined range pass): band pairs wait in LDS and
    // are rechecked after the loop, 64 at a time, one per lane, so that their
    // row loads overlap instead of stalling the wave once per pair (a full
    // queue rechecks in place).  Entry: landmark index in the pass << 40 |
    // settled flag << 32 | point (rank or settled entry).
    const int QCAP = queue_cap(CHUNKED ? a.S : KS, TPS);
    uint64_t *bq = (uint64_t *)(smem + queue_offset(CHUNKED ? a.S : KS, TPS)) + wid * QCAP;
    int qn = 0;                                                    // wave-uniform
    auto flush_queue = [&]() {
        for (int q0 = 0; q0 < qn; q0 += 64) {
            const bool have = q0 + lane < qn;
            const uint64_t e = have ? bq[q0 + lane] : 0ull;
            const int ai = (int)(e >> 40);
            const bool stl = (e >> 32) & 1ull;
            const int64_t p = (int64_t)(uint32_t)e;
            bool memb = false;
            int64_t xo = 0;
            if (have) {
                xo = stl ? (int64_t)gbl(sd.idx)[p] : orig_index(P, p);
                const int32_t lr = A ? A[ai] : ai;
                // a landmark against its own point: s = 0 < e2
                memb = (!stl && lr == p) || exact_member(P, orig_index(P, lr), xo, e2);
            }
            const uint64_t bal = __ballot(memb);
            if (!bal) continue;
            unsigned long long kb = 0;
            if (lane == 0) kb = gatomic_add(o.nkeys, (unsigned long long)__popcll(bal));
            kb = __shfl(kb, 0, 64) + (unsigned long long)mbcnt(bal);
            if (memb) {
                if (kb < o.cap) gbl(o.keys)[kb] = ((uint64_t)(ord0 + ai) << o.bn) | (uint64_t)xo | o.tag;
                if (!stl && o.covered) gatomic_or((unsigned long long *)&o.covered[p >> 6], 1ull << (p & 63));
            }
        }
        qn = 0;
    };
    // Write the key stage out.  Every thread of the workgroup calls it at the
    // same point; after the first barrier no wave appends, so the count is the
    // same for all.
    auto flush_keys = [&]() {
        __syncthreads();
        const int kn = min(*kst_n, kKeyStage);
        if (kn == 0) return;                                        // workgroup-uniform
        if (tid == 0) sh_kbase = gatomic_add(o.nkeys, (unsigned long long)kn);
        __syncthreads();
        const unsigned long long kb = sh_kbase;
        for (int i = tid; i < kn; i += RM_THREADS)
            if (kb + i < o.cap) gbl(o.keys)[kb + i] = kst[i];
        __syncthreads();                                            // every copy has read the stage
        if (tid == 0) *kst_n = 0;
        __syncthreads();
    };
    // One stage: store its staged loads to LDS buffer `buf`, start the loads of
    // the stage two ahead into the same registers, multiply the stage.
    int si = 0;                                                      // stage index (uniform)
    constexpr bool kOneSet = one_set(CHUNKED, KS);
    auto run_stage = [&](int ts, int buf, u32x4 (&pre)[OPS], u32x4 &pre_t) {
        lstore(buf, pre, pre_t);
        __syncthreads();
        gload(ts + (kOneSet ? 1 : 2) * TPS, pre, pre_t);
        if (!CONFLICT) {
            const bool flush = kst_seen[(si + 1) & 1] >= kKeyStage / 2;   // slot (si - 1) & 1: uniform
            if (flush) flush_keys();
            if (tid == 0) kst_seen[si & 1] = flush ? 0 : *kst_n;
            ++si;
        }
        if (!live) return;
      for (int tt = 0; tt < TPS; ++tt) {
        const int t = ts + tt;
        if (t >= t1) break;                                             // wave-uniform
        // resolve: the wave's rows all follow the tile's candidates (i >= j)
        if (CONFLICT && pbase * 32 >= t * 32 + 31) continue;            // wave-uniform
        const int sb = buf * buf_vecs + tt * tile_vecs;                 // this tile's operands in LDS
        const float *thr = (const float *)(sT + buf * THV + tt * 24);   // and thresholds
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

        const float tcut = thr[thr_off + col];
        bool cov = false, slow = false;
        // Fast path: is any pair of the tile possibly a member?  (u, v:
        // conservative thresholds for this point and panel; U, V and aw carry
        // the slack for these two roundings; +inf for padding points.)  The
        // BF16 paths ask it once for both panels (one ballot, one branch); the
        // F16 paths, whose bands are wider, ask it panel by panel.
        bool phit[RM_MP] = {};                                           // per panel (lane)
        if constexpr (!F16) {
            bool hit = false;
#pragma unroll
            for (int pi = 0; pi < RM_MP; ++pi) {
                phit[pi] = false;
                if ((pbase + pi) * 32 >= na) break;                      // wave-uniform
                const f32x16 av = acc[pi];
                float m = fmaxf(fmaxf(av[0], av[1]), av[2]);
                m = fmaxf(fmaxf(m, av[3]), av[4]);
                m = fmaxf(fmaxf(m, av[5]), av[6]);
                m = fmaxf(fmaxf(m, av[7]), av[8]);
                m = fmaxf(fmaxf(m, av[9]), av[10]);
                m = fmaxf(fmaxf(m, av[11]), av[12]);
                m = fmaxf(fmaxf(m, av[13]), av[14]);
                m = fmaxf(m, av[15]);
                phit[pi] = !(m <= (a.refine ? tcut - aw[pi] : tcut));
                hit = hit || phit[pi];
            }
            if (!__ballot(hit)) continue;                                // wave-uniform (a resolve: words stay zero)
        }
#pragma unroll
        for (int pi = 0; pi < RM_MP; ++pi) {
            const int abase = (pbase + pi) * 32;
            if (abase >= na) break;                                      // wave-uniform
            const f32x16 av = acc[pi];
            {
                // this panel alone: no possible member
                bool ph;
                if constexpr (!F16) {
                    ph = phit[pi];
                } else {
                    float m = fmaxf(fmaxf(av[0], av[1]), av[2]);
                    m = fmaxf(fmaxf(m, av[3]), av[4]);
                    m = fmaxf(fmaxf(m, av[5]), av[6]);
                    m = fmaxf(fmaxf(m, av[7]), av[8]);
                    m = fmaxf(fmaxf(m, av[9]), av[10]);
                    m = fmaxf(fmaxf(m, av[11]), av[12]);
                    m = fmaxf(fmaxf(m, av[13]), av[14]);
                    m = fmaxf(m, av[15]);
                    ph = !(m <= (a.refine ? tcut - aw[pi] : tcut));
                }
                if (!__ballot(ph)) continue;                             // (a resolve: words stay zero)
            }
            slow = true;
            const bool stl = t < MT;                                     // wave-uniform
            const int64_t tr = stl ? t : t - MT + RT0;                   // tile in its own array
            const int64_t p = tr * 32 + col;                             // settled entry or rank
            const bool pv = stl ? p < msz : p < n;
            uint32_t mem = 0;
            // the point's original index: for the keys (range pass), or only when a
            // band pair needs the FP64 recheck (resolve)
            const int64_t xo = (!pv || CONFLICT) ? 0 : stl ? (int64_t)gbl(sd.idx)[p] : orig_index(P, p);
            if (a.refine) {
                const float u = thr[col] - aw[pi];
                const float v = thr[32 + col] + aw[pi];
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
                const int bc = __popc(bnd);
                band += (unsigned long long)bc;
                const int bincl = wave_incl_scan(bc);
                const int btot = __shfl(bincl, 63, 64);
                if (!CONFLICT && btot > 0 && qn + btot <= QCAP) {
                    // queue them (rechecked after the loop, lane-parallel)
                    int pos = qn + bincl - bc;
                    while (bnd) {
                        const int i = __builtin_ctz(bnd);
                        bnd &= bnd - 1;
                        const int ai = abase + acc_row(i, half);
                        bq[pos++] = ((uint64_t)ai << 40) | ((uint64_t)(stl ? 1 : 0) << 32) | (uint64_t)(uint32_t)p;
                    }
                    qn += btot;
                    __builtin_amdgcn_wave_barrier();
                } else if (bnd) {
                    // the queue is full (or a resolve): recheck in place
                    const int64_t xr = CONFLICT ? orig_index(P, A[p]) : xo;
                    while (bnd) {
                        const int i = __builtin_ctz(bnd);
                        bnd &= bnd - 1;
                        const int ai = abase + acc_row(i, half);
                        const int32_t lr = A ? A[ai] : ai;
                        if (exact_member(P, orig_index(P, lr), xr, e2)) mem |= 1u << i;
                    }
                }
            } else {
                const float z = thr[64 + col];
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int ai = abase + acc_row(i, half);
                    if (pv && ai < na && (!CONFLICT || ai < p) && av[i] > z) mem |= 1u << i;
                }
            }
            if (CONFLICT) {
                uint32_t w = 0;
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if ((mem >> i) & 1u) w |= 1u << acc_row(i, half);
                w |= __shfl_xor(w, 32, 64);
                if (w != 0u && half == 0 && pv && abase < p) {
                    gbl(T.C32)[p * T.c32_stride + (pbase + pi)] = w;
                    gbl(T.rowflag)[p] = 1;
                }
                continue;
            }
            // append this lane's members to the key stage (one LDS atomic per
            // wave); what does not fit goes to the key buffer directly
            const int cnt = __popc(mem);
            if (!__ballot(cnt != 0)) continue;
            const int incl = wave_incl_scan(cnt);
            const int total = __shfl(incl, 63, 64);
            int lbase = 0;
            if (lane == 0) lbase = atomicAdd(kst_n, total);
            lbase = __shfl(lbase, 0, 64);
            const int spill0 = max(lbase, kKeyStage);                  // first slot past the stage
            const int nspill = lbase + total - spill0;
            unsigned long long gbase = 0;
            if (nspill > 0 && lane == 0) gbase = gatomic_add(o.nkeys, (unsigned long long)nspill);
            gbase = __shfl(gbase, 0, 64);
            cov |= cnt != 0;
            int pos = lbase + incl - cnt;
            while (mem) {
                const int i = __builtin_ctz(mem);
                mem &= mem - 1;
                const uint64_t key = ((uint64_t)(ord0 + abase + acc_row(i, half)) << o.bn) | (uint64_t)xo | o.tag;
                if (pos < kKeyStage) kst[pos] = key;
                else if (gbase + (pos - spill0) < o.cap) gbl(o.keys)[gbase + (pos - spill0)] = key;
                ++pos;
            }
        }
        if (!CONFLICT && slow && o.covered && t >= MT) {                 // wave-uniform
            const int64_t tr = t - MT + RT0;
            const uint64_t m = __ballot(cov);
            const uint64_t bits = (m | (m >> 32)) & 0xffffffffull;
            if (bits && lane == 0)
                gatomic_or((unsigned long long *)&o.covered[(tr * 32) >> 6], (unsigned long long)(bits << ((tr * 32) & 63)));
        }
      }
    };
    // The first stage's loads go out with the setup loads (A operands,
    // accumulator starts); then everything lands before the loop, so the only
    // loads in flight inside it are staging loads and the waitcnt pass need
    // not wait for them before the matrix ops.
    if constexpr (kOneSet) {
        // one register set: a stage stores what the previous one loaded
        gload(t0, preA, pretA);
        __builtin_amdgcn_s_waitcnt(0);
        int ts = t0;
        while (ts + TPS < t1) {
            run_stage(ts, 0, preA, pretA);
            run_stage(ts + TPS, 1, preA, pretA);
            ts += 2 * TPS;
        }
        if (ts < t1) run_stage(ts, 0, preA, pretA);
    } else {
        gload(t0, preA, pretA);
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_sched_barrier(0);       // issue set A before set B: the waits rely on the order
        gload(t0 + TPS, preB, pretB);
        // Unrolled by two (distinct registers), with the odd last stage after the
        // loop: every path into a stage has the set it stores as the older one in flight.
        int ts = t0;
        while (ts + TPS < t1) {
            run_stage(ts, 0, preA, pretA);
            run_stage(ts + TPS, 1, preB, pretB);
            ts += 2 * TPS;
        }
        if (ts < t1) run_stage(ts, 0, preA, pretA);
    }
    if (!CONFLICT && live) flush_queue();
    if (!CONFLICT) flush_keys();
    band = wave_sum(band);
    if (band && lane == 0 && o.st) gatomic_add(&o.st->band, band);
    range_wg_exit<CONFLICT>(T, clk, smem);
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

void range_grid(int na_max, int64_t n_max, int64_t target_wg, int32_t *NGW, int32_t *chunks)
{
    const int npan = (na_max + 31) / 32;
    const int per_wg = RM_WAVES * RM_MP;
    const int ngw = std::max(1, (npan + per_wg - 1) / per_wg);
    const int64_t NT = (n_max + 31) / 32 + 1;                      // + a partial settled tile
    int64_t ch = (target_wg + ngw - 1) / ngw;
    if (ch > NT) ch = NT;
    ch = std::max<int64_t>(8, (ch + 7) / 8 * 8);                  // whole XCD rounds
    *NGW = ngw;
    *chunks = (int32_t)ch;
}

template <int KS, bool F16, bool CONFLICT, bool CHUNKED>
static hipError_t launch_ks(const RangeTask *tasks, const int32_t *task_of, int64_t wgs, int S, int nch,
                            hipStream_t s, LaunchEvents ev)
{
    constexpr int TPS = stage_tiles(CHUNKED, KS);
    // a resolve uses neither the band queue nor the key stage
    const size_t shmem = std::max(CONFLICT ? queue_offset(S, TPS) : range_lds_bytes(S, TPS),
                                  std::max(open_lds_bytes<RM_THREADS>(), accept_lds_bytes<RM_THREADS>()));
    if (shmem + 1024 > kLdsBudget) return hipErrorInvalidValue;
    if (ev.start || ev.stop)          // events attached to the dispatch (not capturable in a graph)
        hipExtLaunchKernelGGL(k_range_mfma<KS, F16, CONFLICT, CHUNKED>, dim3((unsigned)wgs), dim3(RM_THREADS),
                              (uint32_t)shmem, s, ev.start, ev.stop, 0, tasks, task_of, nch, ev.clock);
    else
        k_range_mfma<KS, F16, CONFLICT, CHUNKED><<<dim3((unsigned)wgs), dim3(RM_THREADS), (uint32_t)shmem, s>>>(
            tasks, task_of, nch, ev.clock);
    return hipGetLastError();
}

template <bool F16, bool CONFLICT>
static hipError_t dispatch(const RangeTask *tasks, const int32_t *task_of, int64_t wgs, int S, hipStream_t s,
                           LaunchEvents ev)
{
#define BM_KS(k) launch_ks<k, F16, CONFLICT, false>(tasks, task_of, wgs, S, 1, s, ev)
    switch (S) {
    case 1: return BM_KS(1);
    case 2: return BM_KS(2);
    case 3: return BM_KS(3);
    case 4: return BM_KS(4);
    case 5: return BM_KS(5);
    case 6: return BM_KS(6);
    case 7: return BM_KS(7);
    case 8: return BM_KS(8);
    default: return launch_ks<8, F16, CONFLICT, true>(tasks, task_of, wgs, S, (S + 7) / 8, s, ev);
    }
#undef BM_KS
}

hipError_t launch_range_tasks(const RangeTask *tasks, const int32_t *task_of, int64_t total_wgs, int kind, int S,
                              bool conflict, hipStream_t s, LaunchEvents ev)
{
    if (S < 1 || S > kMaxMfmaSteps) return hipErrorInvalidValue;
    if (total_wgs <= 0) return hipSuccess;
    if (total_wgs > 0x7fffffffLL) return hipErrorInvalidValue;
    const bool f16 = kind == MFMA_F16;
    if (conflict) return f16 ? dispatch<true, true>(tasks, task_of, total_wgs, S, s, ev)
                             : dispatch<false, true>(tasks, task_of, total_wgs, S, s, ev);
    return f16 ? dispatch<true, false>(tasks, task_of, total_wgs, S, s, ev)
               : dispatch<false, false>(tasks, task_of, total_wgs, S, s, ev);
}

} // namespace bm
