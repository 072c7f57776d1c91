// Column-wise encodings and layer schedules, executed in batched form.
//
// The paper gives the column-wise method only as an idea (abstract and
// contributions: an A(m x n).B(n x p) product with each operand as n
// ciphertexts; an h x w image as w column ciphertexts of h slots) plus the
// linearity argument of "Parallelized Matrix Multiplication" and the
// per-channel sums of "Parallelized Convolution Operation".  The schedules:
//
//   matmul  C[idx] = Rescale(Relin(sum_k A_k * Rot(Bbar_k, idx))), idx < P'
//           (RowShifter of "Homomorphic Matrix Multiplication" is a single
//           rotation because P' divides M'; SumColVec becomes the sum over k)
//   conv    Y(c', j') = Rescale(sum_{c,u,v} MulConst(Rot(col(c, s j'+v-pad), u),
//                                K[c'][c][u][v], q_l) + AddConst(bias[c']))
//   square  Rescale(Relin(Tensor(Y, Y)))
//   fc      Z_o = Rescale(sum_{c,j'} MulPlain(Y, W_o,c,j')); Z_o += Rot(Z_o, 2^t);
//           + bias
//
// Batched execution (the same integers as one call per operation):
//   - all ciphertexts of a layer live in one slab [n][ncomp][level+1][N], so
//     every kernel runs once over the whole layer;
//   - one ModUp per input ciphertext is shared by all its rotations
//     (hoisting), and one launch of the inner product per rotation step
//     streams that step's key once for every ciphertext rotated by it;
//   - the MulConst/AddConst accumulation of a whole conv layer is one kernel
//     (each output reads its k*k*C_in rotated inputs, weights held as Shoup
//     pairs), and so is the tensor-accumulate of the matmul and the
//     MulPlain-accumulate of the FC layer.
#include <cmath>
#include <cstring>

#include "slab.h"

namespace vr {

namespace {
constexpr int kThreads = 256;

// value of a tuning knob (0, its default, when never set)
int knob(vr_context* ctx, const char* name)
{
    std::lock_guard<std::mutex> g(ctx->mu);
    auto it = ctx->tuning.find(name);
    return it == ctx->tuning.end() ? 0 : it->second;
}
}  // namespace

Slab new_slab(vr_context* ctx, u32 n, u32 ncomp, u32 level, double scale, hipStream_t s)
{
    Slab sl;
    sl.n = n;
    sl.ncomp = ncomp;
    sl.level = level;
    sl.scale = scale;
    sl.stride = (u64)ncomp * (level + 1) * ctx->n;
    sl.buf = dev_alloc(ctx, std::max<size_t>(1, (size_t)n * sl.stride) * sizeof(u64), s);
    sl.base = as_u64(sl.buf);
    return sl;
}

Slab new_ext_slab(vr_context* ctx, u32 n, u32 level, double scale, hipStream_t s, u32 keep)
{
    if (keep > level) throw Error(VR_EINVAL, "kept limbs above the level");
    Slab sl;
    sl.n = n;
    sl.ncomp = 2;
    sl.level = level;
    sl.ext = 1;
    sl.keep = keep;
    sl.scale = scale;
    sl.stride = (u64)2 * ((keep ? keep : level) + 1 + ctx->K) * ctx->n;
    sl.buf = dev_alloc(ctx, std::max<size_t>(1, (size_t)n * sl.stride) * sizeof(u64), s);
    sl.base = as_u64(sl.buf);
    return sl;
}

constexpr u32 kGatherMax = 64;
struct GatherTable {
    const u64* src[kGatherMax];
};
VR_KERNEL_ARG(GatherTable);

// dst + i * stride <- src[i], i < gridDim.y, as 16-byte pairs
__global__ __launch_bounds__(kThreads) void k_gather_cts(u64* dst, u64 stride, GatherTable t, u32 pairs)
{
    const u32 k = blockIdx.x * kThreads + threadIdx.x;
    if (k >= pairs) return;
    const ulonglong2* src = (const ulonglong2*)t.src[blockIdx.y];
    ((ulonglong2*)(dst + (size_t)blockIdx.y * stride))[k] = src[k];
}

// Uses the ciphertexts in place when they already form a slab, else copies.
Slab gather(vr_context* ctx, const vr_ciphertext* const* cts, u32 n, hipStream_t s)
{
    if (n == 0) throw Error(VR_EINVAL, "empty ciphertext list");
    const vr_ciphertext* c0 = cts[0];
    for (u32 i = 0; i < n; i++) {
        if (!cts[i]) throw Error(VR_EINVAL, "null ciphertext");
        if (cts[i]->level != c0->level) throw Error(VR_ELEVEL, "inputs at different levels");
        if (cts[i]->scale != c0->scale) throw Error(VR_ESCALE, "inputs at different scales");
        if (cts[i]->ncomp != c0->ncomp) throw Error(VR_EINVAL, "inputs with different sizes");
    }
    Slab sl;
    sl.n = n;
    sl.ncomp = c0->ncomp;
    sl.level = c0->level;
    sl.scale = c0->scale;
    sl.stride = (u64)c0->ncomp * (c0->level + 1) * ctx->n;
    bool contiguous = true;
    // in place only within one allocation: separate blocks can sit back to
    // back in the address space, and copies must not span allocations
    for (u32 i = 1; i < n && contiguous; i++)
        contiguous = cts[i]->buf == c0->buf && cts[i]->data == c0->data + (size_t)i * sl.stride;
    if (contiguous) {
        sl.buf = c0->buf;
        sl.base = c0->data;
        return sl;
    }
    sl.buf = dev_alloc(ctx, (size_t)n * sl.stride * sizeof(u64), s);
    sl.base = as_u64(sl.buf);
    // one copy kernel per kGatherMax ciphertexts (their addresses in the
    // arguments) instead of one copy call per ciphertext
    const u32 pairs = (u32)(sl.stride / 2);   // stride is a multiple of N: even
    for (u32 i0 = 0; i0 < n; i0 += kGatherMax) {
        GatherTable t;
        const u32 cnt = std::min(kGatherMax, n - i0);
        for (u32 i = 0; i < cnt; i++) t.src[i] = cts[i0 + i]->data;
        dim3 grid((pairs + kThreads - 1) / kThreads, cnt);
        hipLaunchKernelGGL(k_gather_cts, grid, dim3(kThreads), 0, s, sl.ct(i0), sl.stride, t, pairs);
        VR_CHECK_LAUNCH();
    }
    return sl;
}

void to_handles(vr_context* ctx, const Slab& sl, vr_ciphertext** out)
{
    for (u32 i = 0; i < sl.n; i++) out[i] = view_ct(ctx, sl.buf, sl.ct(i), sl.ncomp, sl.level, sl.scale);
}

namespace {

// ------------------------------------------------------------- kernels

// Input (u, i) packed as u << 24 | i and the weight row pre-multiplied by
// the limb count, so that a block decodes a term with a shift and a mask
// (the scalar unit, not the vector ALU, limits this kernel: a division by
// the column count per term cost more scalar instructions than the products
// cost vector ones).
struct Term {
    u32 in_idx;   // rotation u << 24 | input column index i
    u32 w_idx;    // weight row of filter 0 times the limb count
};
constexpr u32 kTermColBits = 24;

// balanced base-256 digits of x < 2^63 as eight signed bytes (host)
inline u64 balanced_bytes_h(u64 x)
{
    const u64 h = 0x8080808080808080ull;
    return (x + h) ^ h;
}

// For each of n_sets independent image sets s and each output column j':
// out[s][f][j'] = sum_{terms of j'} w_f * in (+ bias on component 0) for every
// filter f, 2 components of nl limbs.  The filters of one column read the
// same inputs, so a block keeps all filters' sums in registers and reads each
// input word once.  Term input (u, j): for u = 0 ciphertext s * n_x + j of
// slab x (stride `stride`, x_limbs limbs per component), for u >= 1
// ciphertext (u - 1) * ustride / rstride + s * n_x + j of slab r (the
// rotations by u of every column of every set, stride `rstride`, nl limbs
// per component).  Output limb l < nk is q_l, limb nk is q_lvl (both read
// from that limb of x), limbs past nk are special primes (modulus l + modoff;
// x contributes nothing): the Q basis is nk = lvl = nl - 1, the extended one
// nk = lvl, and a compact extended one keeps nk < lvl low limbs.
// Term weight offset for filter f and limb l: w_idx + f * w_fstride * nl + l.
//
// Launch order: the logical block id runs over output columns fastest, then
// sets, then rows, then 256-coefficient chunks, so the columns that read the
// same input chunk run back to back; the logical ids are dealt to the 8 XCDs
// in contiguous ranges (hardware hands block b to XCD b mod 8), so those
// blocks share one L2.
//
// Each column's terms come with its rotated terms (u >= 1) first, the
// unrotated ones from rot_end[jo]: the extended basis' special limbs take
// only the rotated terms.  The FP64 path copies its weights (one contiguous
// [term][filter] run per limb and filter group, up to kTermChunk terms at a
// time) into LDS once per block, and each block covers cpb consecutive
// 256-coefficient chunks with them; the products read the weights with
// broadcast LDS loads instead of one scalar load each.
//
// kFp: the instance for the limbs below 2^51 (the others return at once);
// !kFp: 64-bit integer Shoup products for the limbs of 2^51 or more (the
// others return), when k_lincomb_wide does not make them.
constexpr int kMaxFilters = 8;
constexpr u32 kTermChunk = 256;

template <bool kFp>
__global__ __launch_bounds__(kThreads) void k_lincomb(u64* out, u64 out_stride, const u64* x,
                                                      const u64* r, u32 n_x, u32 n_sets, u64 stride,
                                                      u64 rstride, u64 ustride,
                                                      const Term* terms, const u32* term_off,
                                                      const u32* rot_end,
                                                      const u64* w, const u64* ws, const double* wt,
                                                      u32 t_total, u32 w_fstride,
                                                      const u64* bias, u32 nl, u32 nk, u32 lvl, u32 modoff,
                                                      u32 x_limbs, u32 log_n, const ModQ* mq, u32 wo,
                                                      u32 n_filters, u32 total, u32 per_xcd, u32 cpb)
{
    extern __shared__ double wl[];   // [term of the chunk][filter]
    const u32 logical = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (logical >= total) return;   // whole blocks only: no barrier is skipped
    const u32 n = 1u << log_n;
    const u32 chunks = (n + kThreads - 1) / kThreads;
    const u32 jo = logical % wo;
    u32 rest = logical / wo;
    const u32 set = rest % n_sets;
    rest /= n_sets;
    const u32 row = rest % (2 * nl);   // component * nl + limb
    const u32 chunk0 = (rest / (2 * nl)) * cpb;
    const u32 l = row % nl;
    const u64 q = mq[l < nk ? l : l == nk ? lvl : l + modoff].q, q2 = 2 * q;
    const bool x_has = l <= nk;
    const u32 xl = l < nk ? l : lvl;
    const u32 a = term_off[jo], b = x_has ? term_off[jo + 1] : rot_end[jo];
    const u32 n_out = n_filters * wo;
    const u64* xb = x + (size_t)set * n_x * stride;
    const u64* rb = r + (size_t)set * n_x * rstride;
    const size_t fst = (size_t)w_fstride * nl;
    constexpr u32 kColMask = (1u << kTermColBits) - 1;
    if (kFp) {
        if (q >= (1ull << 51)) return;   // whole blocks: no barrier is skipped
        // FP64 products (the block's limb has one modulus): inputs and
        // weights balanced, each product within 0.75 q, the sums reduced
        // every four terms (below 3.5 q < 2^53)
        const double qd = (double)q, qinv = 1.0 / qd;
        for (u32 f0 = 0, g = 0; f0 < n_filters; f0 += kMaxFilters, g++) {
            const u32 nf = min((u32)kMaxFilters, n_filters - f0);
            const double* wg = wt + (size_t)(g * nl + l) * t_total * kMaxFilters;
            u32 loaded = 0xffffffffu;   // first term of the chunk held in LDS
            for (u32 cc = 0; cc < cpb && chunk0 + cc < chunks; cc++) {
                const u32 t = (chunk0 + cc) * kThreads + threadIdx.x;
                const bool active = t < n;
                const size_t tile = (size_t)row * n + t;
                const size_t xtile = ((size_t)(row / nl) * x_limbs + (x_has ? xl : 0)) * n + t;
                double acc[kMaxFilters];
#pragma unroll
                for (int f = 0; f < kMaxFilters; f++) acc[f] = 0;
                for (u32 c0 = a; c0 < b; c0 += kTermChunk) {
                    const u32 ce = min(b, c0 + kTermChunk);
                    if (c0 != loaded) {
                        __syncthreads();   // readers of the previous chunk are done
                        for (u32 i = threadIdx.x; i < (ce - c0) * kMaxFilters; i += kThreads)
                            wl[i] = wg[(size_t)c0 * kMaxFilters + i];
                        __syncthreads();
                        loaded = c0;
                    }
                    for (u32 k0 = c0; k0 < ce; k0 += 8) {
                        u64 xv[8];
#pragma unroll
                        for (int i = 0; i < 8; i++) {
                            if (k0 + i < ce) {
                                const Term tm = terms[k0 + i];
                                const u32 u = tm.in_idx >> kTermColBits, j = tm.in_idx & kColMask;
                                xv[i] = !active ? 0
                                        : u == 0 ? xb[(size_t)j * stride + xtile]
                                                 : rb[(u - 1) * ustride + (size_t)j * rstride + tile];
                            }
                        }
#pragma unroll
                        for (int i = 0; i < 8; i++) {
                            if (k0 + i < ce) {
                                const double xf = to_bal(xv[i], q, qd);
                                const double* wk = wl + (k0 + i - c0) * kMaxFilters;
#pragma unroll
                                for (int f = 0; f < kMaxFilters; f++)
                                    if (f < (int)nf) acc[f] += fmulmod(xf, wk[f], qd, qinv);
                            }
                            if ((i & 3) == 3) {
#pragma unroll
                                for (int f = 0; f < kMaxFilters; f++) acc[f] = fbal(acc[f], qd, qinv);
                            }
                        }
                    }
                }
                if (!active) continue;
#pragma unroll
                for (int f = 0; f < kMaxFilters; f++) {
                    if (f < (int)nf) {
                        const u32 o = (f0 + f) * wo + jo;
                        double v = acc[f];
                        if (bias && row < nl) v += to_bal(bias[(size_t)o * nl + l], q, qd);
                        out[(size_t)(set * n_out + o) * out_stride + tile] = to_canon(v, qd, qinv);
                    }
                }
            }
        }
        return;
    }
    // integer path (limbs of 2^51 or more): no barrier, scalar weight loads
    if (q < (1ull << 51)) return;
    for (u32 cc = 0; cc < cpb && chunk0 + cc < chunks; cc++) {
        const u32 t = (chunk0 + cc) * kThreads + threadIdx.x;
        if (t >= n) break;
        const size_t tile = (size_t)row * n + t;
        const size_t xtile = ((size_t)(row / nl) * x_limbs + (x_has ? xl : 0)) * n + t;
        for (u32 f0 = 0; f0 < n_filters; f0 += kMaxFilters) {
            const u32 nf = min((u32)kMaxFilters, n_filters - f0);
            u64 acc[kMaxFilters];
#pragma unroll
            for (int f = 0; f < kMaxFilters; f++) acc[f] = 0;
            // eight terms at a time: their input words are loaded together so the
            // loads overlap instead of each waiting on the previous one
            for (u32 k0 = a; k0 < b; k0 += 8) {
                u64 xv[8];
                u32 wrow[8];
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    if (k0 + i < b) {
                        const Term tm = terms[k0 + i];
                        const u32 u = tm.in_idx >> kTermColBits, j = tm.in_idx & kColMask;
                        xv[i] = u == 0 ? xb[(size_t)j * stride + xtile] : rb[(u - 1) * ustride + (size_t)j * rstride + tile];
                        wrow[i] = tm.w_idx;
                    }
                }
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    if (k0 + i < b) {
#pragma unroll
                        for (int f = 0; f < kMaxFilters; f++) {
                            if (f < (int)nf) {
                                const size_t wi = wrow[i] + (f0 + f) * fst + l;
                                u64 v = acc[f] + shoup_lazy(xv[i], w[wi], ws[wi], q);
                                acc[f] = v >= q2 ? v - q2 : v;
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int f = 0; f < kMaxFilters; f++) {
                if (f < (int)nf) {
                    const u32 o = (f0 + f) * wo + jo;
                    u64 v = acc[f];
                    if (bias && row < nl) v += bias[(size_t)o * nl + l];
                    v = v >= q2 ? v - q2 : v;
                    v = v >= q ? v - q : v;
                    out[(size_t)(set * n_out + o) * out_stride + tile] = v;
                }
            }
        }
    }
}

// The rows of k_lincomb whose modulus is 2^51 or more (the 60-bit q_0, wide
// special primes; every such q below 2^63), as exact FP64 sums instead of
// 64-bit integer products.  Input word x and weight w (canonical residues)
// are split into 21-bit pieces, x = x_0 + x_1 2^21 + x_2 2^42 and likewise
// w, so x w = sum_m 2^(21 m) S_m with S_m = sum_{i+j=m} x_i w_j: nine
// products below 2^42, summed exactly in five doubles per filter (below 2^50
// over kWideChunk terms).  At the end of each chunk of terms the sums fold
// into a residue: S_0 + 2^21 S_1 + 2^42 S_2 as a 128-bit value reduced mod
// q, S_3 and S_4 times 2^63 and 2^84 mod q.  The weight pieces of a chunk
// ([term][filter][piece], kWideChunk terms) sit in LDS.  Block order and
// term ranges as in k_lincomb; the rows are (component, wide limb) pairs,
// the wide limbs the set bits of wide_mask.
constexpr u32 kWidePieces = 3, kWideChunk = 85;   // 85 x 8 x 3 doubles: 16320 bytes

__global__ __launch_bounds__(kThreads) void k_lincomb_wide(u64* out, u64 out_stride, const u64* x,
                                                           const u64* r, u32 n_x, u32 n_sets, u64 stride,
                                                           u64 rstride, u64 ustride, const Term* terms,
                                                           const u32* term_off, const u32* rot_end,
                                                           const double* wp, u32 t_total, const u64* bias,
                                                           u32 nl, u32 nk, u32 lvl, u32 modoff, u32 x_limbs,
                                                           u32 log_n, const ModQ* mq, u32 wo, u32 n_filters,
                                                           u64 wide_mask, u32 n_wide, u32 total, u32 per_xcd,
                                                           u32 cpb)
{
    extern __shared__ double wl[];   // [term of the chunk][filter][piece]
    const u32 logical = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (logical >= total) return;   // whole blocks only: no barrier is skipped
    const u32 n = 1u << log_n;
    const u32 chunks = (n + kThreads - 1) / kThreads;
    const u32 jo = logical % wo;
    u32 rest = logical / wo;
    const u32 set = rest % n_sets;
    rest /= n_sets;
    const u32 wrow = rest % (2 * n_wide);
    const u32 chunk0 = (rest / (2 * n_wide)) * cpb;
    const u32 wi = wrow % n_wide;
    u64 bits = wide_mask;
    for (u32 i = 0; i < wi; i++) bits &= bits - 1;
    const u32 l = (u32)__ffsll((unsigned long long)bits) - 1;
    const u32 row = (wrow / n_wide) * nl + l;
    const ModQ m = mq[l < nk ? l : l == nk ? lvl : l + modoff];
    const u64 c3 = reduce128(0, 1ull << 63, m), c4 = reduce128(1ull << 20, 0, m);
    const bool x_has = l <= nk;
    const u32 xl = l < nk ? l : lvl;
    const u32 a = term_off[jo], b = x_has ? term_off[jo + 1] : rot_end[jo];
    const u32 n_out = n_filters * wo;
    const u64* xb = x + (size_t)set * n_x * stride;
    const u64* rb = r + (size_t)set * n_x * rstride;
    constexpr u32 kColMask = (1u << kTermColBits) - 1;
    constexpr u64 kPiece = (1ull << 21) - 1;
    constexpr u32 kRun = kMaxFilters * kWidePieces;   // doubles per term
    for (u32 f0 = 0, g = 0; f0 < n_filters; f0 += kMaxFilters, g++) {
        const u32 nf = min((u32)kMaxFilters, n_filters - f0);
        const double* wg = wp + (size_t)(g * n_wide + wi) * t_total * kRun;
        u32 loaded = 0xffffffffu;
        for (u32 cc = 0; cc < cpb && chunk0 + cc < chunks; cc++) {
            const u32 t = (chunk0 + cc) * kThreads + threadIdx.x;
            const bool active = t < n;
            const size_t tile = (size_t)row * n + t;
            const size_t xtile = ((size_t)(row / nl) * x_limbs + (x_has ? xl : 0)) * n + t;
            u64 acc[kMaxFilters];
#pragma unroll
            for (int f = 0; f < kMaxFilters; f++) acc[f] = 0;
            for (u32 c0 = a; c0 < b; c0 += kWideChunk) {
                const u32 ce = min(b, c0 + kWideChunk);
                if (c0 != loaded) {
                    __syncthreads();
                    for (u32 i = threadIdx.x; i < (ce - c0) * kRun; i += kThreads) wl[i] = wg[(size_t)c0 * kRun + i];
                    __syncthreads();
                    loaded = c0;
                }
                double S[kMaxFilters][5];
#pragma unroll
                for (int f = 0; f < kMaxFilters; f++)
#pragma unroll
                    for (int k = 0; k < 5; k++) S[f][k] = 0;
                for (u32 k0 = c0; k0 < ce; k0 += 4) {
                    u64 xv[4];
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        xv[i] = 0;
                        if (k0 + i < ce && active) {
                            const Term tm = terms[k0 + i];
                            const u32 u = tm.in_idx >> kTermColBits, j = tm.in_idx & kColMask;
                            xv[i] = u == 0 ? xb[(size_t)j * stride + xtile]
                                           : rb[(u - 1) * ustride + (size_t)j * rstride + tile];
                        }
                    }
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        if (k0 + i < ce) {
                            const double x0 = u2f(xv[i] & kPiece), x1 = u2f((xv[i] >> 21) & kPiece),
                                         x2 = u2f(xv[i] >> 42);
                            const double* wk = wl + (k0 + i - c0) * kRun;
#pragma unroll
                            for (int f = 0; f < kMaxFilters; f++) {
                                if (f < (int)nf) {
                                    const double w0 = wk[f * 3], w1 = wk[f * 3 + 1], w2 = wk[f * 3 + 2];
                                    S[f][0] = __fma_rn(x0, w0, S[f][0]);
                                    S[f][1] = __fma_rn(x1, w0, __fma_rn(x0, w1, S[f][1]));
                                    S[f][2] = __fma_rn(x2, w0, __fma_rn(x1, w1, __fma_rn(x0, w2, S[f][2])));
                                    S[f][3] = __fma_rn(x2, w1, __fma_rn(x1, w2, S[f][3]));
                                    S[f][4] = __fma_rn(x2, w2, S[f][4]);
                                }
                            }
                        }
                    }
                }
#pragma unroll
                for (int f = 0; f < kMaxFilters; f++) {
                    if (f < (int)nf) {
                        const u64 s0 = f2u(S[f][0]), s1 = f2u(S[f][1]), s2 = f2u(S[f][2]);
                        const u64 l1 = s1 << 21, l2 = s2 << 42;
                        u64 lo = s0 + l1;
                        u64 hi = (s1 >> 43) + (s2 >> 22) + (lo < l1 ? 1 : 0);
                        lo += l2;
                        hi += lo < l2 ? 1 : 0;
                        u64 v = reduce128(hi, lo, m);
                        v = add_mod(v, mul_mod(f2u(S[f][3]), c3, m), m.q);
                        v = add_mod(v, mul_mod(f2u(S[f][4]), c4, m), m.q);
                        acc[f] = add_mod(acc[f], v, m.q);
                    }
                }
            }
            if (!active) continue;
#pragma unroll
            for (int f = 0; f < kMaxFilters; f++) {
                if (f < (int)nf) {
                    const u32 o = (f0 + f) * wo + jo;
                    u64 v = acc[f];
                    if (bias && row < nl) v = add_mod(v, bias[(size_t)o * nl + l], m.q);
                    out[(size_t)(set * n_out + o) * out_stride + tile] = v;
                }
            }
        }
    }
}

// The conv's weighted sums on the matrix cores, exactly.  Per output limb
// (modulus q), column j' and filter f the sum is sum_k x_k w_{f,k} mod q over
// the column's terms k.  Each input word x_k < 2^63 is written in balanced
// base 256, x_k = sum_a x_{k,a} 2^(8a) with signed digits, and the host
// writes each w'_{f,k,a} = 2^(8a) w_{f,k} mod q in balanced base 256 too,
// w' = sum_j d_{f,k,a,j} 2^(8j).  Then sum_k x_k w_{f,k} = sum_j 2^(8j) S_{f,j}
// (mod q) with S_{f,j} = sum_{k,a} x_{k,a} d_{f,k,a,j}: an int8 dot product
// (|S| < 2^31 for up to 16384 terms).  One v_mfma_i32_16x16x32_i8 takes 4
// terms x 8 digits a on K and 16 coefficients on N; its 16 rows are
// 4 filters x 4 digits j, and the four tiles T = 2h + e hold filters
// 4h + 0..3 with j = 4e + 0..3, so that a lane's accumulators hold all eight
// S_{f,j} of filters f = g and g + 4 (g = lane / 16) for its coefficient.
// It folds them into a residue: in FP64 below 2^51 (three exact partial
// sums, two of them times 2^24 and 2^48 mod q), else as a signed 128-bit
// value reduced mod q.
//
// Table: lane l of (filter group, limb, K-step s, tile T) holds row
// rho = l % 16 (filter 4h + rho / 4, digit j = 4e + rho % 4) for term
// 4s + l / 16 of the column; byte a is d_{f,k,a,j}.  Columns with the same
// weight rows share one table (col_at[j'] its offset).  Each wave covers 64
// coefficients (four N-tiles) per pass with the weight words of a step held
// across them; block order as in k_lincomb.  The block's term sources (the
// input or rotated limb row each term reads) sit in LDS, up to kMfmaSrcChunk
// terms at a time, and each wave loads the next step's input words while the
// current step's products run.  Occupancy floors: 4 waves per SIMD for the
// FP64-fold instance (127 VGPRs), 3 for the 128-bit one (a few bytes spill).
typedef int v4i __attribute__((ext_vector_type(4)));
constexpr u32 kMfmaMaxTerms = 16384;
constexpr u32 kMfmaSrcChunk = 512;

__device__ __forceinline__ u64 bal_bytes(u64 x)
{
    const u64 h = 0x8080808080808080ull;
    return (x + h) ^ h;
}

template <bool kFp>
__global__ __launch_bounds__(kThreads, kFp ? 4 : 3) void k_lincomb_mfma(u64* out, u64 out_stride, const u64* x, const u64* r,
                                                           u32 n_x, u32 n_sets, u64 stride, u64 rstride,
                                                           u64 ustride, const Term* terms, const u32* term_off,
                                                           const u32* rot_end, const u64* at, const u64* col_at, const u64* kc,
                                                           const u64* bias, u32 nl, u32 nk, u32 lvl, u32 modoff,
                                                           u32 x_limbs, u32 log_n, const ModQ* mq, u32 wo,
                                                           u32 n_filters, u32 total, u32 per_xcd, u32 cpb)
{
    const u32 logical = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (logical >= total) return;
    const u32 n = 1u << log_n;
    const u32 passes = n / kThreads;
    const u32 jo = logical % wo;
    u32 rest = logical / wo;
    const u32 set = rest % n_sets;
    rest /= n_sets;
    const u32 row = rest % (2 * nl);
    const u32 pass0 = (rest / (2 * nl)) * cpb;
    const u32 l = row % nl;
    const ModQ m = mq[l < nk ? l : l == nk ? lvl : l + modoff];
    const u64 q = m.q;
    const bool x_has = l <= nk;
    const u32 xl = l < nk ? l : lvl;
    const u32 a = term_off[jo];
    const u32 n_all = term_off[jo + 1] - a;
    const u32 n_use = x_has ? n_all : rot_end[jo] - a;   // special limbs: rotated terms only
    const u32 steps_all = (n_all + 3) / 4, steps = (n_use + 3) / 4;
    const u32 n_out = n_filters * wo;
    const u64* xb = x + (size_t)set * n_x * stride;
    const u64* rb = r + (size_t)set * n_x * rstride;
    constexpr u32 kColMask = (1u << kTermColBits) - 1;
    const u32 lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const u32 g = lane >> 4, col = lane & 15;
    // kFp: the rows below 2^51 (FP64 fold), else the others
    if (kFp != (q < (1ull << 51))) return;
    const double qd = (double)q, qinv = 1.0 / qd;
    // 2^24, 2^48 mod q (balanced) for the FP64 fold; 2^128 mod q for the
    // sign of the 128-bit fold (the plan's table, per limb)
    const double c24b = to_bal(kc[3 * l], q, qd), c48b = to_bal(kc[3 * l + 1], q, qd);
    const u64 c128 = kc[3 * l + 2];
    const size_t xrow = ((size_t)(row / nl) * x_limbs + (x_has ? xl : 0)) * n;
    const size_t orow = (size_t)row * n;
    // term k's limb row (null past the column's terms), for terms
    // held_at .. held_at + kMfmaSrcChunk - 1
    __shared__ const u64* srcs[kMfmaSrcChunk];
    u32 held_at = 0xffffffffu;
    for (u32 f0 = 0, grp = 0; f0 < n_filters; f0 += kMaxFilters, grp++) {
        const u64* tab = at + col_at[jo] + ((size_t)grp * nl + l) * steps_all * 256 + lane;
        for (u32 cc = 0; cc < cpb && pass0 + cc < passes; cc++) {
            const u32 base = (pass0 + cc) * kThreads + wave * 64 + col;   // N-tile nt adds 16 nt
            v4i acc[4][4];
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int T = 0; T < 4; T++) acc[i][T] = v4i{0, 0, 0, 0};
            for (u32 k0 = 0; k0 < 4 * steps; k0 += kMfmaSrcChunk) {
                const u32 kn = min(4 * steps - k0, kMfmaSrcChunk);   // a multiple of 4
                if (k0 != held_at) {
                    __syncthreads();
                    for (u32 i = threadIdx.x; i < kn; i += kThreads) {
                        const u32 k = k0 + i;
                        const u64* src = nullptr;
                        if (k < n_use) {
                            const Term tm = terms[a + k];
                            const u32 u = tm.in_idx >> kTermColBits, j = tm.in_idx & kColMask;
                            src = u == 0 ? xb + (size_t)j * stride + xrow
                                         : rb + (u - 1) * ustride + (size_t)j * rstride + orow;
                        }
                        srcs[i] = src;
                    }
                    __syncthreads();
                    held_at = k0;
                }
                const u32 s0 = k0 / 4, s1 = s0 + kn / 4;
                long cur[4] = {0, 0, 0, 0};
                if (const u64* src = srcs[g]) {
#pragma unroll
                    for (int i = 0; i < 4; i++) cur[i] = (long)src[base + 16 * i];
                }
                for (u32 s = s0; s < s1; s++) {
                    long w[4];
#pragma unroll
                    for (int T = 0; T < 4; T++) w[T] = (long)tab[((size_t)s * 4 + T) * 64];
                    long nxt[4] = {0, 0, 0, 0};
                    if (s + 1 < s1) {
                        if (const u64* src = srcs[4 * (s + 1 - s0) + g]) {
#pragma unroll
                            for (int i = 0; i < 4; i++) nxt[i] = (long)src[base + 16 * i];
                        }
                    }
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        const long b = (long)bal_bytes((u64)cur[i]);
#pragma unroll
                        for (int T = 0; T < 4; T++)
                            acc[i][T] = __builtin_amdgcn_mfma_i32_16x16x32_i8(w[T], b, acc[i][T], 0, 0, 0);
                    }
#pragma unroll
                    for (int i = 0; i < 4; i++) cur[i] = nxt[i];
                }
            }
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const u32 coef = base + 16 * i;
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const u32 f = f0 + 4 * h + g;
                    if (f >= n_filters) continue;
                    const v4i lo4 = acc[i][2 * h], hi4 = acc[i][2 * h + 1];
                    const u32 o = f * wo + jo;
                    u64 v;
                    if (kFp) {
#pragma clang fp contract(off)
                        const double A0 = __fma_rn((double)lo4[2], 65536.0, __fma_rn((double)lo4[1], 256.0, (double)lo4[0]));
                        const double A1 = __fma_rn((double)hi4[1], 65536.0, __fma_rn((double)hi4[0], 256.0, (double)lo4[3]));
                        const double A2 = __fma_rn((double)hi4[3], 256.0, (double)hi4[2]);
                        double t = fbal(fmulmod(A1, c24b, qd, qinv) + fmulmod(A2, c48b, qd, qinv), qd, qinv) + A0;
                        if (bias && row < nl) t += to_bal(bias[(size_t)o * nl + l], q, qd);
                        v = to_canon(t, qd, qinv);
                    } else {
                        const i64 Plo = (i64)lo4[0] + ((i64)lo4[1] << 8) + ((i64)lo4[2] << 16) + ((i64)lo4[3] << 24);
                        const i64 Phi = (i64)hi4[0] + ((i64)hi4[1] << 8) + ((i64)hi4[2] << 16) + ((i64)hi4[3] << 24);
                        // V = Plo + Phi 2^32 in two's complement 128 bits
                        const u64 x1 = (u64)Phi << 32;
                        u64 lo = (u64)Plo + x1;
                        u64 hi = (u64)(Plo >> 63) + (u64)(Phi >> 32) + (lo < x1 ? 1 : 0);
                        v = reduce128(hi, lo, m);
                        if ((i64)hi < 0) v = sub_mod(v, c128, q);   // the value read as 2^128 + V
                        if (bias && row < nl) v = add_mod(v, bias[(size_t)o * nl + l], q);
                    }
                    out[(size_t)(set * n_out + o) * out_stride + orow + coef] = v;
                }
            }
        }
    }
}

// T = sum_k A_k (x) R_k: 3-component tensor accumulate over n_terms pairs
__global__ __launch_bounds__(kThreads) void k_tensor_acc(u64* T, const u64* A, u64 a_stride,
                                                         const u64* R, u64 r_stride, u32 n_terms,
                                                         u32 nl, u32 log_n, const ModQ* mq, u32 accumulate)
{
    const u32 n = 1u << log_n;
    const u32 t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    const u32 l = blockIdx.y;
    const ModQ m = mq[l];
    const size_t poly = (size_t)nl * n, off = (size_t)l * n + t;
    u64 d0 = 0, d1 = 0, d2 = 0;
    if (accumulate) d0 = T[off], d1 = T[poly + off], d2 = T[2 * poly + off];
    for (u32 k = 0; k < n_terms; k++) {
        const u64* a = A + (size_t)k * a_stride + off;
        const u64* r = R + (size_t)k * r_stride + off;
        u64 a0 = a[0], a1 = a[poly], b0 = r[0], b1 = r[poly];
        d0 = add_mod(d0, mul_mod(a0, b0, m), m.q);
        d1 = add_mod(d1, add_mod(mul_mod(a0, b1, m), mul_mod(a1, b0, m), m.q), m.q);
        d2 = add_mod(d2, mul_mod(a1, b1, m), m.q);
    }
    T[off] = d0;
    T[poly + off] = d1;
    T[2 * poly + off] = d2;
}

// out_c (3 comps) = tensor(a_c, b_c) for n_ct ciphertext pairs
__global__ __launch_bounds__(kThreads) void k_tensor_batch(u64* out, const u64* a, const u64* b,
                                                           u64 in_stride, u32 nl, u32 log_n,
                                                           const ModQ* mq)
{
    const u32 n = 1u << log_n;
    const u32 t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    const u32 l = blockIdx.y % nl, c = blockIdx.y / nl;
    const ModQ m = mq[l];
    const size_t poly = (size_t)nl * n, off = (size_t)l * n + t;
    const u64* x = a + (size_t)c * in_stride + off;
    const u64* y = b + (size_t)c * in_stride + off;
    u64* o = out + (size_t)c * 3 * poly + off;
    u64 a0 = x[0], a1 = x[poly], b0 = y[0], b1 = y[poly];
    o[0] = mul_mod(a0, b0, m);
    o[poly] = add_mod(mul_mod(a0, b1, m), mul_mod(a1, b0, m), m.q);
    o[2 * poly] = mul_mod(a1, b1, m);
}

// out[o] = sum_i Y_i * P[o][i] for outputs o0 .. o0 + kFcGroup - 1 (o0 =
// blockIdx.z * kFcGroup): one thread per (limb, coefficient) accumulates both
// components of every output of its group, so each plaintext word is read
// once and each input word once per group.  Plaintext (o, i) starts at
// P + (o * n_in + i) * p_stride, limbs [N] each.
constexpr int kFcGroup = 8;

// Compact copy of evaluation-domain limbs that repeat in runs of 2^rep
// consecutive words: out[v][u] = in[v][u 2^rep]; *bad = 1 when a run holds
// two different words (then the copy is not used).
__global__ __launch_bounds__(kThreads) void k_compact_runs(const u64* in, u64* out, u32 log_n, u32 rep, int* bad)
{
    const size_t n = (size_t)1 << log_n, cn = n >> rep;
    const size_t u = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (u >= cn) return;
    const u64* src = in + (size_t)blockIdx.y * n + (u << rep);
    const u64 v0 = src[0];
    bool same = true;
    for (u32 k = 1; k < (1u << rep); k++) same = same && src[k] == v0;
    if (!same) atomicOr(bad, 1);
    out[(size_t)blockIdx.y * cn + u] = v0;
}

// FC weight products of the x^2 tensors (lazy relinearisation): for outputs
// o0 .. o0 + kSqfcGroup - 1 (o0 = blockIdx.z * kSqfcGroup) and limb l,
//   out_o = sum_i (y_i0^2, 2 y_i0 y_i1, y_i1^2) P[o][i]     (3 components),
// the tensor of each input formed once per limb and output group (groups of
// five: the ten classes of the paper's networks take two, and the smaller
// accumulator set leaves more waves per SIMD).  A block covers 64
// coefficients; its four waves take every fourth input each and their
// residues are summed through LDS at the end.  kFp: the limbs below 2^51, as
// exact FP64 products (balanced operands, sums reduced every four inputs);
// otherwise 128-bit integer sums (the others return at once).
constexpr int kSqfcGroup = 5;
constexpr u32 kSqfcWaves = 4;

template <bool kFp>
__global__ __launch_bounds__(kThreads) void k_sqfc_acc(u64* out, u64 out_stride, const u64* Y, u64 y_stride,
                                                       u64 y_comp, u32 n_in, const u64* P, u64 p_stride,
                                                       u32 n_out, u32 nl, u32 log_n, const ModQ* mq, u32 rep)
{
    __shared__ u64 red[kSqfcWaves - 1][kSqfcGroup][64];
    const u32 n = 1u << log_n;
    const u32 lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const u32 t = blockIdx.x * 64 + lane;   // n is a multiple of 64
    const u32 l = blockIdx.y;
    const u32 o0 = blockIdx.z * kSqfcGroup;
    const u32 cnt = min((u32)kSqfcGroup, n_out - o0);
    const ModQ m = mq[l];
    if (kFp != (m.q < (1ull << 51))) return;   // whole blocks: no barrier is skipped
    const size_t off0 = (size_t)l * n + t, yoff1 = y_comp + off0;
    const size_t poff = (size_t)l * (n >> rep) + (t >> rep);   // weights: runs of 2^rep words kept once
    const u64* Pg = P + (size_t)o0 * n_in * p_stride + poff;
    u64 res[3][kSqfcGroup];   // this wave's residues
    if (kFp) {
        const double qd = (double)m.q, qinv = 1.0 / qd;
        double acc[3][kSqfcGroup];
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int g = 0; g < kSqfcGroup; g++) acc[c][g] = 0;
        u32 k = 0;
        // the next input's words load while this one is summed
        u64 n0 = wave < n_in ? Y[(size_t)wave * y_stride + off0] : 0;
        u64 n1 = wave < n_in ? Y[(size_t)wave * y_stride + yoff1] : 0;
        for (u32 i = wave; i < n_in; i += kSqfcWaves, k++) {
            const double y0 = to_bal(n0, m.q, qd);
            const double y1 = to_bal(n1, m.q, qd);
            if (i + kSqfcWaves < n_in) {
                n0 = Y[(size_t)(i + kSqfcWaves) * y_stride + off0];
                n1 = Y[(size_t)(i + kSqfcWaves) * y_stride + yoff1];
            }
            const double x01 = fmulmod(y0, y1, qd, qinv);
            // the tensor balanced again (|d| <= q / 2 + 1): each weight
            // product within 0.75 q
            const double d[3] = {fbal(fmulmod(y0, y0, qd, qinv), qd, qinv), fbal(x01 + x01, qd, qinv),
                                 fbal(fmulmod(y1, y1, qd, qinv), qd, qinv)};
#pragma unroll
            for (int g = 0; g < kSqfcGroup; g++) {
                if (g < (int)cnt) {
                    const double p = to_bal(Pg[((size_t)g * n_in + i) * p_stride], m.q, qd);
#pragma unroll
                    for (int c = 0; c < 3; c++) acc[c][g] += fmulmod(d[c], p, qd, qinv);
                }
            }
            if ((k & 3) == 3) {   // below 3.5 q < 2^53
#pragma unroll
                for (int c = 0; c < 3; c++)
#pragma unroll
                    for (int g = 0; g < kSqfcGroup; g++) acc[c][g] = fbal(acc[c][g], qd, qinv);
            }
        }
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int g = 0; g < kSqfcGroup; g++) res[c][g] = to_canon(acc[c][g], qd, qinv);
    } else {
        u64 h[3][kSqfcGroup], lo[3][kSqfcGroup];
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int g = 0; g < kSqfcGroup; g++) h[c][g] = lo[c][g] = 0;
        u32 k = 0;
        u64 n0 = wave < n_in ? Y[(size_t)wave * y_stride + off0] : 0;
        u64 n1 = wave < n_in ? Y[(size_t)wave * y_stride + yoff1] : 0;
        for (u32 i = wave; i < n_in; i += kSqfcWaves, k++) {
            const u64 y0 = n0, y1 = n1;
            if (i + kSqfcWaves < n_in) {
                n0 = Y[(size_t)(i + kSqfcWaves) * y_stride + off0];
                n1 = Y[(size_t)(i + kSqfcWaves) * y_stride + yoff1];
            }
            const u64 x01 = mul_mod(y0, y1, m);
            const u64 d[3] = {mul_mod(y0, y0, m), add_mod(x01, x01, m.q), mul_mod(y1, y1, m)};
#pragma unroll
            for (int g = 0; g < kSqfcGroup; g++) {
                if (g < (int)cnt) {
                    const u64 p = Pg[((size_t)g * n_in + i) * p_stride];
#pragma unroll
                    for (int c = 0; c < 3; c++) mac128(h[c][g], lo[c][g], d[c], p);
                }
            }
            if ((k & 31) == 31) {   // keep every 128-bit sum below 2^127
#pragma unroll
                for (int c = 0; c < 3; c++)
#pragma unroll
                    for (int g = 0; g < kSqfcGroup; g++) {
                        lo[c][g] = reduce128(h[c][g], lo[c][g], m);
                        h[c][g] = 0;
                    }
            }
        }
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int g = 0; g < kSqfcGroup; g++) res[c][g] = reduce128(h[c][g], lo[c][g], m);
    }
    // sum the waves' residues, one component at a time
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (wave > 0) {
#pragma unroll
            for (int g = 0; g < kSqfcGroup; g++) red[wave - 1][g][lane] = res[c][g];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int g = 0; g < kSqfcGroup; g++) {
                if (g < (int)cnt) {
                    u64 v = res[c][g];
#pragma unroll
                    for (u32 w = 0; w + 1 < kSqfcWaves; w++) v = add_mod(v, red[w][g][lane], m.q);
                    out[(size_t)(o0 + g) * out_stride + (size_t)c * nl * n + off0] = v;
                }
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void k_mulplain_acc(u64* out, u64 out_stride,
                                                           const u64* Y, u64 y_stride, u64 y_comp,
                                                           u32 n_in, const u64* P, u64 p_stride,
                                                           u32 n_out, u32 nl, u32 log_n, const ModQ* mq,
                                                           u32 rep)
{
    const u32 n = 1u << log_n;
    const u32 t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    const u32 l = blockIdx.y;
    const u32 o0 = blockIdx.z * kFcGroup;
    const u32 cnt = min((u32)kFcGroup, n_out - o0);
    const ModQ m = mq[l];
    u64 h0[kFcGroup], l0[kFcGroup], h1[kFcGroup], l1[kFcGroup];
#pragma unroll
    for (int g = 0; g < kFcGroup; g++) h0[g] = l0[g] = h1[g] = l1[g] = 0;
    // output limbs [2][nl][N]; input component 1 at y_comp (the inputs may
    // hold more limbs than the nl read here)
    const size_t off0 = (size_t)l * n + t, off1 = (size_t)(nl + l) * n + t, yoff1 = y_comp + off0;
    const size_t poff = (size_t)l * (n >> rep) + (t >> rep);   // weights: runs of 2^rep words kept once
    for (u32 i = 0; i < n_in; i++) {
        const u64 y0 = Y[(size_t)i * y_stride + off0];
        const u64 y1 = Y[(size_t)i * y_stride + yoff1];
#pragma unroll
        for (int g = 0; g < kFcGroup; g++) {
            if (g < (int)cnt) {
                const u64 p = P[((size_t)(o0 + g) * n_in + i) * p_stride + poff];
                mac128(h0[g], l0[g], y0, p);
                mac128(h1[g], l1[g], y1, p);
            }
        }
        if ((i & 31) == 31) {   // keep every 128-bit sum below 2^127
#pragma unroll
            for (int g = 0; g < kFcGroup; g++) {
                l0[g] = reduce128(h0[g], l0[g], m);
                l1[g] = reduce128(h1[g], l1[g], m);
                h0[g] = h1[g] = 0;
            }
        }
    }
#pragma unroll
    for (int g = 0; g < kFcGroup; g++) {
        if (g < (int)cnt) {
            u64* o = out + (size_t)(o0 + g) * out_stride;
            o[off0] = reduce128(h0[g], l0[g], m);
            o[off1] = reduce128(h1[g], l1[g], m);
        }
    }
}

// Key-switching scratch per ciphertext (ModUp digits, coefficient copy,
// inner-product sums, ModDown scratch); layer calls switch at most
// kSwitchBudget bytes' worth of ciphertexts at a time so that a layer of any
// size runs in bounded memory (at N = 2^16, l = 24 that is ~120 ciphertexts).
constexpr size_t kSwitchBudget = size_t(16) << 30;

// key ranges must tile [0, n) in order
void check_ranges(const std::vector<KeyRange>& keys, u32 n)
{
    u32 at = 0;
    for (const KeyRange& kr : keys) {
        if (kr.begin != at || kr.end < kr.begin || !kr.ek) throw Error(VR_EINVAL, "key ranges must tile the slab");
        at = kr.end;
    }
    if (at != n) throw Error(VR_EINVAL, "key ranges must tile the slab");
}

u32 switch_chunk(vr_context* ctx, u32 level, u32 n_ct)
{
    KsShape k = ks_shape(ctx, level);
    const size_t per = ((size_t)k.beta * k.next + k.nq + 2 * k.next + 2 * (ctx->K + k.nq)) * ctx->n * 8;
    size_t c = std::max<size_t>(1, kSwitchBudget / per);
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        auto it = ctx->tuning.find("switch_chunk");
        if (it != ctx->tuning.end() && it->second > 0) c = (size_t)it->second;
    }
    return (u32)std::min<size_t>(c, n_ct);
}

// Rotations of every ciphertext of `in` by every step; out[si] is a slab of
// in.n rotated ciphertexts (step si).  One ModUp per input (hoisting), one
// inner-product launch per step, chunk of inputs and key range (ciphertexts
// [begin, end) of `in` switch with the keys of their range's session), one
// ModDown per step and chunk whatever the sessions.
void rotate_slab_keyed(vr_context* ctx, const std::vector<KeyRange>& keys, const Slab& in,
                       const std::vector<int32_t>& steps, std::vector<Slab>& out, hipStream_t s)
{
    const u32 level = in.level, n_ct = in.n;
    const size_t n = ctx->n;
    KsShape k = ks_shape(ctx, level);
    check_ranges(keys, n_ct);
    std::vector<u32> gs;
    for (int32_t st : steps) {
        u32 g = galois_element(ctx, st);
        if (g != 1)
            for (const KeyRange& kr : keys) (void)rot_key(kr.ek, g);
        gs.push_back(g);
    }
    const u32 cs = switch_chunk(ctx, level, n_ct);
    const u64 xs = (u64)k.beta * k.next * n, us = (u64)2 * k.next * n;
    BufPtr xbuf = dev_alloc(ctx, ((size_t)cs * xs + (size_t)cs * k.nq * n) * sizeof(u64), s);
    u64* X = as_u64(xbuf);
    u64* coef = X + (size_t)cs * xs;
    BufPtr ubuf = dev_alloc(ctx, ((size_t)cs * us + keyswitch_moddown_scratch(ctx, level, cs)) * sizeof(u64), s);
    u64* U = as_u64(ubuf);
    u64* md = U + (size_t)cs * us;
    out.clear();
    // every step's output in one allocation: step si at all.base + si * n_ct * stride
    Slab all = new_slab(ctx, n_ct * (u32)steps.size(), 2, level, in.scale, s);
    for (size_t si = 0; si < steps.size(); si++) {
        Slab r = all;
        r.n = n_ct;
        r.base = all.base + si * n_ct * all.stride;
        out.push_back(r);
    }
    for (u32 c0 = 0; c0 < n_ct; c0 += cs) {
        const u32 nc = std::min(cs, n_ct - c0);
        const u64* src = in.ct(c0);
        keyswitch_modup_batch(ctx, src + (size_t)k.nq * n, in.stride, nc, level, X, coef, s);
        for (size_t si = 0; si < steps.size(); si++) {
            u64* dst = out[si].ct(c0);
            if (gs[si] == 1) {
                VR_HIP(hipMemcpyAsync(dst, src, (size_t)nc * in.stride * sizeof(u64), hipMemcpyDeviceToDevice, s));
            } else {
                for (const KeyRange& kr : keys) {
                    const u32 lo = std::max(kr.begin, c0), hi = std::min(kr.end, c0 + nc);
                    if (lo >= hi) continue;
                    keyswitch_inner_batch(ctx, X + (size_t)(lo - c0) * xs, xs, in.ct(lo) + (size_t)k.nq * n,
                                          in.stride, hi - lo, rot_key(kr.ek, gs[si]).data, level, gs[si],
                                          U + (size_t)(lo - c0) * us, us, s);
                }
                keyswitch_moddown_batch(ctx, U, us, nc, level, dst, dst + (size_t)k.nq * n, all.stride, src,
                                        gs[si], nullptr, in.stride, md, s);
            }
        }
    }
}

void rotate_slab(vr_context* ctx, const vr_eval_keys* ek, const Slab& in,
                 const std::vector<int32_t>& steps, std::vector<Slab>& out, hipStream_t s)
{
    rotate_slab_keyed(ctx, {KeyRange{0, in.n, ek}}, in, steps, out, s);
}

// The rotations of rotate_slab_keyed without their ModDown: out[si] is an
// extended slab holding, per ciphertext, P times its rotation by steps[si]
// (the key-switch sums of sigma_g(ModUp(c1)) with P sigma_g(c0) folded into
// component 0's Q limbs by the inner-product kernel).  Steps must not be 0
// mod the slot count.  keep > 0: only the limbs of a compact extended slab
// (q_0..q_{keep-1}, q_level, the special primes) are made.
void rotate_slab_ext(vr_context* ctx, const std::vector<KeyRange>& keys, const Slab& in,
                     const std::vector<int32_t>& steps, std::vector<Slab>& out, hipStream_t s, u32 keep)
{
    const u32 level = in.level, n_ct = in.n;
    const size_t n = ctx->n;
    if (in.ext || in.ncomp != 2) throw Error(VR_EINVAL, "rotation needs 2-component ciphertexts");
    KsShape k = ks_shape(ctx, level);
    check_ranges(keys, n_ct);
    std::vector<u32> gs;
    for (int32_t st : steps) {
        u32 g = galois_element(ctx, st);
        if (g == 1) throw Error(VR_EINVAL, "extended rotation by 0");
        for (const KeyRange& kr : keys) (void)rot_key(kr.ek, g);
        gs.push_back(g);
    }
    const u32 cs = switch_chunk(ctx, level, n_ct);
    const u64 xs = (u64)k.beta * k.next * n;
    BufPtr xbuf = dev_alloc(ctx, ((size_t)cs * xs + (size_t)cs * k.nq * n) * sizeof(u64), s);
    u64* X = as_u64(xbuf);
    u64* coef = X + (size_t)cs * xs;
    out.clear();
    Slab all = new_ext_slab(ctx, n_ct * (u32)steps.size(), level, in.scale, s, keep);
    for (size_t si = 0; si < steps.size(); si++) {
        Slab r = all;
        r.n = n_ct;
        r.base = all.base + si * n_ct * all.stride;
        out.push_back(r);
    }
    for (u32 c0 = 0; c0 < n_ct; c0 += cs) {
        const u32 nc = std::min(cs, n_ct - c0);
        keyswitch_modup_batch(ctx, in.ct(c0) + (size_t)k.nq * n, in.stride, nc, level, X, coef, s, keep);
        // the steps two at a time: each digit word read once for both
        for (size_t si = 0; si < steps.size(); si += 2)
            for (const KeyRange& kr : keys) {
                const u32 lo = std::max(kr.begin, c0), hi = std::min(kr.end, c0 + nc);
                if (lo >= hi) continue;
                if (si + 1 < steps.size())
                    keyswitch_inner_batch2(ctx, X + (size_t)(lo - c0) * xs, xs, in.ct(lo) + (size_t)k.nq * n,
                                           in.stride, hi - lo, rot_key(kr.ek, gs[si]).data,
                                           rot_key(kr.ek, gs[si + 1]).data, level, gs[si], gs[si + 1],
                                           out[si].ct(lo), out[si + 1].ct(lo), all.stride, s, in.ct(lo), in.stride,
                                           keep);
                else
                    keyswitch_inner_batch(ctx, X + (size_t)(lo - c0) * xs, xs, in.ct(lo) + (size_t)k.nq * n,
                                          in.stride, hi - lo, rot_key(kr.ek, gs[si]).data, level, gs[si],
                                          out[si].ct(lo), all.stride, s, in.ct(lo), in.stride, keep);
            }
    }
}

// ModDown by P q_l of every ciphertext of an extended slab: level l - 1,
// scale / q_l (chunked so the conversion scratch stays bounded)
Slab mod_down_rescale_slab(vr_context* ctx, const Slab& in, hipStream_t s)
{
    if (!in.ext) throw Error(VR_EINVAL, "ModDown by P q_l needs an extended slab");
    const u32 level = in.level;
    if (level == 0) throw Error(VR_ELEVEL, "no limb left to rescale by");
    const size_t n = ctx->n;
    const u32 no = in.keep ? in.keep : level;   // output limbs
    Slab out = new_slab(ctx, in.n, 2, no - 1, in.scale / (double)ctx->mod[level], s);
    const u32 cs = switch_chunk(ctx, level, in.n);
    BufPtr md = dev_alloc(ctx, keyswitch_moddown_scratch(ctx, level, cs) * sizeof(u64), s);
    for (u32 c0 = 0; c0 < in.n; c0 += cs) {
        const u32 nc = std::min(cs, in.n - c0);
        u64* o = out.ct(c0);
        keyswitch_moddown_rescale_batch(ctx, in.ct(c0), in.stride, nc, level, o, o + (size_t)no * n, out.stride,
                                        nullptr, nullptr, 0, as_u64(md), s, in.keep);
    }
    return out;
}

// relinearise a slab of 3-component ciphertexts into 2-component ones, each
// key range with its session's relinearisation key; with `rescale` the
// ModDown also divides by q_l (one rounding, level l - 1, scale / q_l)
Slab relin_slab_keyed(vr_context* ctx, const std::vector<KeyRange>& keys, const Slab& T, hipStream_t s,
                      bool rescale)
{
    const u32 level = T.level, n_ct = T.n;
    if (rescale && level == 0) throw Error(VR_ELEVEL, "no limb left to rescale by");
    const size_t n = ctx->n;
    KsShape k = ks_shape(ctx, level);
    check_ranges(keys, n_ct);
    const u32 cs = switch_chunk(ctx, level, n_ct);
    const u64 xs = (u64)k.beta * k.next * n, us = (u64)2 * k.next * n;
    BufPtr xbuf = dev_alloc(ctx, ((size_t)cs * xs + (size_t)cs * k.nq * n) * sizeof(u64), s);
    u64* X = as_u64(xbuf);
    BufPtr ubuf = dev_alloc(ctx, ((size_t)cs * us + keyswitch_moddown_scratch(ctx, level, cs)) * sizeof(u64), s);
    u64* U = as_u64(ubuf);
    Slab out = rescale ? new_slab(ctx, n_ct, 2, level - 1, T.scale / (double)ctx->mod[level], s)
                       : new_slab(ctx, n_ct, 2, level, T.scale, s);
    const size_t out_comp = (size_t)(rescale ? level : level + 1) * n;
    for (u32 c0 = 0; c0 < n_ct; c0 += cs) {
        const u32 nc = std::min(cs, n_ct - c0);
        const u64* t = T.ct(c0);
        keyswitch_modup_batch(ctx, t + (size_t)2 * k.nq * n, T.stride, nc, level, X, X + (size_t)cs * xs, s);
        for (const KeyRange& kr : keys) {
            const u32 lo = std::max(kr.begin, c0), hi = std::min(kr.end, c0 + nc);
            if (lo >= hi) continue;
            keyswitch_inner_batch(ctx, X + (size_t)(lo - c0) * xs, xs, T.ct(lo) + (size_t)2 * k.nq * n, T.stride,
                                  hi - lo, kr.ek->rlk.data, level, 1, U + (size_t)(lo - c0) * us, us, s);
        }
        u64* o = out.ct(c0);
        if (rescale)
            keyswitch_moddown_rescale_batch(ctx, U, us, nc, level, o, o + out_comp, out.stride, t,
                                            t + (size_t)k.nq * n, T.stride, U + (size_t)cs * us, s);
        else
            keyswitch_moddown_batch(ctx, U, us, nc, level, o, o + out_comp, out.stride, t, 1,
                                    t + (size_t)k.nq * n, T.stride, U + (size_t)cs * us, s);
    }
    return out;
}

Slab relin_slab(vr_context* ctx, const vr_eval_keys* ek, const Slab& T, hipStream_t s)
{
    return relin_slab_keyed(ctx, {KeyRange{0, T.n, ek}}, T, s, false);
}

Slab relin_rescale_slab(vr_context* ctx, const vr_eval_keys* ek, const Slab& T, hipStream_t s)
{
    return relin_slab_keyed(ctx, {KeyRange{0, T.n, ek}}, T, s, true);
}

Slab rescale_slab(vr_context* ctx, const Slab& in, hipStream_t s)
{
    if (in.level == 0) throw Error(VR_ELEVEL, "no limb left to rescale by");
    Slab out = new_slab(ctx, in.n, in.ncomp, in.level - 1, in.scale / (double)ctx->mod[in.level], s);
    rescale_dense(ctx, in.base, out.base, in.n * in.ncomp, in.level, s);
    return out;
}

// Sums of ct x ct tensor products for the encrypted-weight layers: output z
// (group g = z / n_sub, term list z mod n_sub) is
//   sum_t Tensor(A(term_a[t]), B + g b_group + term_b[t])   (3 components),
// A(o) = A1 + (o & ~top) when the top bit of o is set, else A0 + o (word
// offsets); a_comp / b_comp are the operands' component strides.
__global__ __launch_bounds__(kThreads) void k_tensor_terms(u64* out, u64 out_stride, const u64* A0, const u64* A1,
                                                           const u64* B, u64 b_group, const u64* term_a,
                                                           const u64* term_b, const u32* term_off, u32 n_sub,
                                                           u32 nl, u64 a_comp, u64 b_comp, u32 log_n,
                                                           const ModQ* mq)
{
    const u32 n = 1u << log_n;
    const u32 t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    const u32 l = blockIdx.y, z = blockIdx.z;
    const u32 g = z / n_sub, sub = z - g * n_sub;
    const ModQ m = mq[l];
    const size_t off = (size_t)l * n + t;
    const u64* Bg = B + (size_t)g * b_group;
    u64 d0 = 0, d1 = 0, d2 = 0;
    for (u32 k = term_off[sub]; k < term_off[sub + 1]; k++) {
        const u64 ao = term_a[k];
        const u64* a = ((ao >> 63) ? A1 + (ao & ~(1ull << 63)) : A0 + ao) + off;
        const u64* b = Bg + term_b[k] + off;
        const u64 a0 = a[0], a1 = a[a_comp], b0 = b[0], b1 = b[b_comp];
        d0 = add_mod(d0, mul_mod(a0, b0, m), m.q);
        d1 = add_mod(d1, add_mod(mul_mod(a0, b1, m), mul_mod(a1, b0, m), m.q), m.q);
        d2 = add_mod(d2, mul_mod(a1, b1, m), m.q);
    }
    u64* o = out + (size_t)z * out_stride + off;
    const size_t oc = (size_t)nl * n;
    o[0] = d0;
    o[oc] = d1;
    o[2 * oc] = d2;
}

// Dense layer on neuron ciphertexts: out_o = sum_j W[o][j] Z_j (+ bias_o on
// every slot of c0), W[o][j] as exact residues [RHA(W q_l)]_{q_i} at
// wq + (o n_in + j) nl + l, bias residues at bq + o nl + l.
__global__ __launch_bounds__(kThreads) void k_dense(u64* out, u64 out_stride, const u64* Z, u64 z_stride,
                                                    u32 n_in, const u64* wq, const u64* bq, u32 nl, u32 log_n,
                                                    const ModQ* mq)
{
    const u32 n = 1u << log_n;
    const u32 t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    const u32 comp = blockIdx.y / nl, l = blockIdx.y % nl, o = blockIdx.z;
    const ModQ m = mq[l];
    const size_t off = ((size_t)comp * nl + l) * n + t;
    u64 acc = comp == 0 ? bq[(size_t)o * nl + l] : 0;
    for (u32 j = 0; j < n_in; j++)
        acc = add_mod(acc, mul_mod(wq[((size_t)o * n_in + j) * nl + l], Z[(size_t)j * z_stride + off], m), m.q);
    out[(size_t)o * out_stride + off] = acc;
}

// the slab's ciphertexts on their first nl limbs (a level drop keeps the message)
Slab drop_slab(vr_context* ctx, const Slab& x, u32 level, hipStream_t s)
{
    if (level == x.level) return x;
    Slab y = new_slab(ctx, x.n, x.ncomp, level, x.scale, s);
    const size_t w = (size_t)(level + 1) * ctx->n * sizeof(u64);
    VR_HIP(hipMemcpy2DAsync(y.base, w, x.base, (size_t)(x.level + 1) * ctx->n * sizeof(u64), w,
                            (size_t)x.n * x.ncomp, hipMemcpyDeviceToDevice, s));
    return y;
}

// AddConst c on every ciphertext of a slab (c0 gets [RHA(c scale)]_{q_l})
void add_const_slab(vr_context* ctx, const Slab& x, double c, hipStream_t s)
{
    LimbConsts k;
    for (u32 l = 0; l <= x.level; l++) k.c[l] = double_to_mod(c * x.scale, ctx->mod[l]);
    for (u32 i = 0; i < x.n; i++) launch_add_scalar(ctx, x.ct(i), x.ct(i), x.level + 1, k, s);
}

// sum_i coeffs[i] x^i by Horner's rule (degree d >= 1, depth d): t =
// Rescale(MulConst(x, a_d; q_l) + a_{d-1}), then t = Rescale(Relin(Tensor(t,
// x dropped to t's level))) + a_i for i = d-2 .. 0.
Slab poly_slab(vr_context* ctx, const vr_eval_keys* ek, const Slab& x, const double* coeffs, u32 d,
               hipStream_t s)
{
    if (x.ncomp != 2) throw Error(VR_EINVAL, "polynomial inputs must be 2-component");
    if (d < 1) throw Error(VR_EINVAL, "degree must be at least 1");
    if (x.level < d) throw Error(VR_ELEVEL, "not enough levels for the polynomial's depth");
    const u32 lv = x.level;
    const double dq = (double)ctx->mod[lv];
    LimbConsts k;
    for (u32 l = 0; l <= lv; l++) {
        k.c[l] = double_to_mod(coeffs[d] * dq, ctx->mod[l]);
        k.cs[l] = shoup_companion(k.c[l], ctx->mod[l]);
    }
    Slab t = new_slab(ctx, x.n, 2, lv, x.scale * dq, s);
    launch_mul_scalar(ctx, t.base, x.base, 2 * x.n, lv + 1, k, s);
    add_const_slab(ctx, t, coeffs[d - 1], s);
    t = rescale_slab(ctx, t, s);
    for (int i = (int)d - 2; i >= 0; i--) {
        Slab xd = drop_slab(ctx, x, t.level, s);
        Slab P = new_slab(ctx, x.n, 3, t.level, t.scale * xd.scale, s);
        dim3 grid((ctx->n + kThreads - 1) / kThreads, x.n * (t.level + 1));
        {
            ProfScope prof(ctx, kProfTensor, s, (u64)x.n * 2 * (t.level + 1));
            hipLaunchKernelGGL(k_tensor_batch, grid, dim3(kThreads), 0, s, P.base, t.base, xd.base, t.stride,
                               t.level + 1, ctx->log_n, ctx->d_modq);
            VR_CHECK_LAUNCH();
        }
        t = relin_rescale_slab(ctx, ek, P, s);
        add_const_slab(ctx, t, coeffs[i], s);
    }
    return t;
}

Slab dense_slab(vr_context* ctx, const Slab& z, const double* W, const double* bias, u32 n_out, hipStream_t s)
{
    if (z.ncomp != 2) throw Error(VR_EINVAL, "dense inputs must be 2-component");
    if (z.level < 1) throw Error(VR_ELEVEL, "dense needs a level to rescale");
    const u32 nl = z.level + 1, n_in = z.n;
    const double dq = (double)ctx->mod[z.level];
    Slab acc = new_slab(ctx, n_out, 2, z.level, z.scale * dq, s);
    std::vector<u64> h((size_t)n_out * n_in * nl + (size_t)n_out * nl);
    for (u32 o = 0; o < n_out; o++)
        for (u32 j = 0; j < n_in; j++)
            for (u32 l = 0; l < nl; l++)
                h[((size_t)o * n_in + j) * nl + l] = double_to_mod(W[(size_t)o * n_in + j] * dq, ctx->mod[l]);
    u64* hb = h.data() + (size_t)n_out * n_in * nl;
    for (u32 o = 0; o < n_out; o++)
        for (u32 l = 0; l < nl; l++) hb[(size_t)o * nl + l] = double_to_mod(bias[o] * acc.scale, ctx->mod[l]);
    BufPtr tab = dev_alloc(ctx, h.size() * sizeof(u64), s);
    VR_HIP(hipMemcpyAsync(tab->ptr, h.data(), h.size() * sizeof(u64), hipMemcpyHostToDevice, s));
    dim3 grid((ctx->n + kThreads - 1) / kThreads, 2 * nl, n_out);
    hipLaunchKernelGGL(k_dense, grid, dim3(kThreads), 0, s, acc.base, acc.stride, z.base, z.stride, n_in,
                       as_u64(tab), as_u64(tab) + (size_t)n_out * n_in * nl, nl, ctx->log_n, ctx->d_modq);
    VR_CHECK_LAUNCH();
    // the host table must outlive the asynchronous copy
    VR_HIP(hipStreamSynchronize(s));
    return rescale_slab(ctx, acc, s);
}

// Encrypted-weight layers: the products summed per output, one
// relinearisation and rescale for all outputs, then the bias ciphertexts
// (one level lower, at the rescaled scale) added.
Slab tensor_terms_slab(vr_context* ctx, const Slab& x, const Slab* rot_all, const Slab& W, u64 w_group,
                       const std::vector<u64>& ta, const std::vector<u64>& tb, const std::vector<u32>& toff,
                       u32 n_sub, u32 n_out, hipStream_t s)
{
    if (W.level != x.level) throw Error(VR_ELEVEL, "weight ciphertexts must sit at the inputs' level");
    const u32 nl = x.level + 1;
    Slab T = new_slab(ctx, n_out, 3, x.level, x.scale * W.scale, s);
    BufPtr tab = dev_alloc(ctx, (ta.size() + tb.size()) * sizeof(u64) + toff.size() * sizeof(u32), s);
    u64* dta = as_u64(tab);
    u64* dtb = dta + ta.size();
    u32* doff = (u32*)(dtb + tb.size());
    VR_HIP(hipMemcpyAsync(dta, ta.data(), ta.size() * sizeof(u64), hipMemcpyHostToDevice, s));
    VR_HIP(hipMemcpyAsync(dtb, tb.data(), tb.size() * sizeof(u64), hipMemcpyHostToDevice, s));
    VR_HIP(hipMemcpyAsync(doff, toff.data(), toff.size() * sizeof(u32), hipMemcpyHostToDevice, s));
    dim3 grid((ctx->n + kThreads - 1) / kThreads, nl, n_out);
    {
        ProfScope prof(ctx, kProfTensor, s, (u64)n_out * 2 * nl);
        hipLaunchKernelGGL(k_tensor_terms, grid, dim3(kThreads), 0, s, T.base, T.stride, x.base,
                           rot_all ? rot_all->base : x.base, W.base, w_group, dta, dtb, doff, n_sub, nl,
                           (u64)nl * ctx->n, (u64)nl * ctx->n, ctx->log_n, ctx->d_modq);
        VR_CHECK_LAUNCH();
    }
    VR_HIP(hipStreamSynchronize(s));   // the host term tables must outlive their copies
    return T;
}

void add_bias_cts(vr_context* ctx, const Slab& y, const Slab& bias, u32 per_bias, hipStream_t s)
{
    if (bias.level != y.level) throw Error(VR_ELEVEL, "bias ciphertexts must sit one level below the weights");
    if (bias.scale != y.scale) throw Error(VR_ESCALE, "bias ciphertexts must carry the rescaled products' scale");
    if (bias.ncomp != 2) throw Error(VR_EINVAL, "bias ciphertexts must be 2-component");
    for (u32 i = 0; i < y.n; i++)
        launch_addsub(ctx, y.ct(i), y.ct(i), bias.ct(i / per_bias), 2, y.level + 1, false, s);
}

Slab conv_encw_slab(vr_context* ctx, const vr_eval_keys* ek, const Slab& x, u32 C_in, u32 w, u32 pad,
                    const Slab& Kw, const Slab& Bias, u32 C_out, u32 k, u32 stride, hipStream_t s)
{
    if (x.ncomp != 2 || Kw.ncomp != 2) throw Error(VR_EINVAL, "inputs and weights must be 2-component");
    if (Kw.n != C_out * C_in * k * k || Bias.n != C_out) throw Error(VR_EINVAL, "weight or bias count");
    const u32 wo = (w + 2 * pad - k) / stride + 1;
    std::vector<int32_t> steps;
    for (u32 u = 1; u < k; u++) steps.push_back((int32_t)u);
    std::vector<Slab> rot;
    if (!steps.empty()) rotate_slab(ctx, ek, x, steps, rot, s);
    const u32 n_x = C_in * w;
    std::vector<u64> ta, tb;
    std::vector<u32> toff{0};
    for (u32 jo = 0; jo < wo; jo++) {
        for (u32 c = 0; c < C_in; c++)
            for (u32 v = 0; v < k; v++) {
                const int jj = (int)(stride * jo + v) - (int)pad;
                if (jj < 0 || jj >= (int)w) continue;
                for (u32 u = 0; u < k; u++) {
                    const u64 col = (u64)c * w + (u32)jj;
                    ta.push_back(u == 0 ? col * x.stride
                                        : ((u64)1 << 63) | (((u64)(u - 1) * n_x + col) * x.stride));
                    tb.push_back((((u64)c * k + u) * k + v) * Kw.stride);
                }
            }
        toff.push_back((u32)ta.size());
    }
    Slab T = tensor_terms_slab(ctx, x, rot.empty() ? nullptr : &rot[0], Kw, (u64)C_in * k * k * Kw.stride, ta,
                               tb, toff, wo, C_out * wo, s);
    rot.clear();
    Slab y = relin_rescale_slab(ctx, ek, T, s);
    add_bias_cts(ctx, y, Bias, wo, s);
    return y;
}

Slab fc_encw_slab(vr_context* ctx, const vr_eval_keys* ek, const Slab& y, const Slab& Wc, const Slab& Bias,
                  u32 n_out, u32 block, hipStream_t s)
{
    if (Wc.n != n_out * y.n || Bias.n != n_out) throw Error(VR_EINVAL, "weight or bias count");
    std::vector<u64> ta, tb;
    std::vector<u32> toff{0};
    for (u32 i = 0; i < y.n; i++) {
        ta.push_back((u64)i * y.stride);
        tb.push_back((u64)i * Wc.stride);
    }
    toff.push_back((u32)ta.size());
    Slab T = tensor_terms_slab(ctx, y, nullptr, Wc, (u64)y.n * Wc.stride, ta, tb, toff, 1, n_out, s);
    Slab z = relin_rescale_slab(ctx, ek, T, s);
    for (u32 st = 1; st < block; st <<= 1) {
        std::vector<Slab> r;
        rotate_slab(ctx, ek, z, {(int32_t)st}, r, s);
        launch_addsub(ctx, z.base, z.base, r[0].base, z.n * 2, z.level + 1, false, s);
    }
    add_bias_cts(ctx, z, Bias, 1, s);
    return z;
}

Slab square_slab(vr_context* ctx, const vr_eval_keys* ek, const Slab& in, hipStream_t s)
{
    if (in.ncomp != 2) throw Error(VR_EINVAL, "square needs 2-component inputs");
    const u32 nl = in.level + 1;
    Slab T = new_slab(ctx, in.n, 3, in.level, in.scale * in.scale, s);
    dim3 grid((ctx->n + kThreads - 1) / kThreads, in.n * nl);
    {
        ProfScope prof(ctx, kProfTensor, s, (u64)in.n * 2 * nl);
        hipLaunchKernelGGL(k_tensor_batch, grid, dim3(kThreads), 0, s, T.base, in.base, in.base,
                           in.stride, nl, ctx->log_n, ctx->d_modq);
        VR_CHECK_LAUNCH();
    }
    return relin_rescale_slab(ctx, ek, T, s);
}

u32 pow2ceil(u32 x)
{
    u32 p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Device-resident constants of one conv layer call: weights [RHA(K q_l)]_{q_i}
// with Shoup companions (one row per (c', c, u, v)), the AddConst value per
// output and limb, and the term list (input index, weight row of filter 0)
// per output column.  Input (u, c, j) is u << 24 | (c * w + j).
struct ConvPlan {
    BufPtr buf;
    const Term* terms = nullptr;
    const u32* off = nullptr;
    const u32* rot_end = nullptr;   // per column: first unrotated term
    const u64 *w = nullptr, *ws = nullptr, *bias = nullptr;
    // balanced FP64 weights per filter group g, limb l and term t (global
    // index), filter f: wt[((g nl + l) t_total + t) 8 + f] (moduli below 2^51)
    const double* wt = nullptr;
    // 21-bit pieces of the canonical weights on the limbs of 2^51 or more
    // (the set bits of wide_mask, n_wide of them):
    // wp[(((g n_wide + wi) t_total + t) 8 + f) 3 + j]; none when a wide
    // modulus reaches 2^63 or nl exceeds 64 (k_lincomb's integer path then)
    const double* wp = nullptr;
    u64 wide_mask = 0;
    u32 n_wide = 0;
    bool any_wide = false;   // some limb's modulus is 2^51 or more
    // matrix-core tables (k_lincomb_mfma), one per distinct column pattern;
    // col_at[j'] the offset of column j''s; absent when too large; kc per
    // limb: 2^24, 2^48 and 2^128 mod q
    const u64* at = nullptr;
    const u64* col_at = nullptr;
    const u64* kc = nullptr;
    u32 t_total = 0, max_col = 0;   // terms in all, most terms of one column
};

// P mod q (host)
u64 p_mod_h(vr_context* ctx, u64 q)
{
    u64 v = 1 % q;
    for (u32 k = 0; k < ctx->K; k++) v = (u64)((u128)v * (ctx->mod[ctx->L + 1 + k] % q) % q);
    return v;
}

// The conv's weight and bias tables over nl limbs: q_0..q_level, and with
// `ext` also p_0..p_{K-1} for the lazy-ModDown form, where the unrotated
// terms (u = 0) and the bias act on P times the input (P w on the Q limbs,
// nothing on the special ones) and the rotated terms on the rotations'
// key-switch sums (w on every limb).
const ConvPlan& conv_plan(vr_context* ctx, u32 C_in, u32 w, u32 pad, const double* K,
                          const double* bias, u32 C_out, u32 k, u32 stride, u32 level, double out_scale,
                          bool ext, u32 keep)
{
    // limbs as k_lincomb maps them: q_0..q_{nk-1}, q_level, then the special
    // primes when ext (nk = keep for a compact extended basis, else level)
    const u32 wo = (w + 2 * pad - k) / stride + 1, nk = ext && keep ? keep : level;
    const u32 nl = ext ? nk + 1 + ctx->K : level + 1;
    const size_t nw = (size_t)C_out * C_in * k * k;
    if ((size_t)C_in * w >= (1u << kTermColBits) || k >= 256 || nw * nl >= (1ull << 32))
        throw Error(VR_EINVAL, "conv layer too large: C_in * w must stay below 2^24, k below 256");
    std::string key = ext ? "convx:" : "conv:";
    u32 shape[8] = {C_in, w, pad, C_out, k, stride, level, ext ? keep : 0u};
    key.append((const char*)shape, sizeof shape);
    key.append((const char*)&out_scale, sizeof out_scale);
    key.append((const char*)K, nw * sizeof(double));
    key.append((const char*)bias, C_out * sizeof(double));
    std::lock_guard<std::mutex> g(ctx->mu);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) return *(const ConvPlan*)it->second.get();

    const double dq = (double)ctx->mod[level];
    std::vector<u64> wv(nw * nl), wsv(nw * nl), bv((size_t)C_out * wo * nl);
    std::vector<double> wfv(nw * nl);
    auto mod_of = [&](u32 l) { return l < nk ? l : l == nk ? level : ctx->L + 1 + (l - nk - 1); };
    for (size_t r = 0; r < nw; r++)
        for (u32 l = 0; l < nl; l++) {
            const u64 q = ctx->mod[mod_of(l)];
            u64 v = double_to_mod(K[r] * dq, q);
            if (ext && (r / k) % k == 0)   // unrotated term: P w on Q limbs, none on P limbs
                v = l <= nk ? (u64)((u128)v * p_mod_h(ctx, q) % q) : 0;
            wv[r * nl + l] = v;
            wsv[r * nl + l] = shoup_companion(v, q);
            wfv[r * nl + l] = v > q / 2 ? -(double)(q - v) : (double)v;
        }
    for (u32 co = 0; co < C_out; co++)
        for (u32 l = 0; l < nl; l++) {
            const u64 q = ctx->mod[mod_of(l)];
            u64 b = l <= nk ? double_to_mod(bias[co] * out_scale, q) : 0;
            if (ext && l <= nk) b = (u64)((u128)b * p_mod_h(ctx, q) % q);
            for (u32 jo = 0; jo < wo; jo++) bv[((size_t)co * wo + jo) * nl + l] = b;
        }
    // one term list per output column, weight rows of filter 0 (filter c'
    // adds c' * C_in * k * k): the rotated terms (u >= 1) first, the
    // unrotated ones from rot_end[jo]
    std::vector<Term> terms;
    std::vector<u32> off(1, 0), rot_end;
    for (u32 jo = 0; jo < wo; jo++) {
        for (int pass = 0; pass < 2; pass++) {
            if (pass == 1) rot_end.push_back((u32)terms.size());
            for (u32 c = 0; c < C_in; c++)
                for (u32 v = 0; v < k; v++) {
                    int jj = (int)(stride * jo + v) - (int)pad;
                    if (jj < 0 || jj >= (int)w) continue;
                    for (u32 u = pass ? 0 : 1; u < (pass ? 1 : k); u++)
                        terms.push_back({(u32)(((size_t)u << kTermColBits) | ((size_t)c * w + jj)),
                                         (u32)((((size_t)c * k + u) * k + v) * nl)});
                }
        }
        off.push_back((u32)terms.size());
    }
    // the FP64 weights as contiguous [term][filter] runs per group and limb
    const u32 groups = (C_out + kMaxFilters - 1) / kMaxFilters, t_total = (u32)terms.size();
    const size_t fst = (size_t)C_in * k * k * nl;
    std::vector<double> wtv((size_t)groups * nl * t_total * kMaxFilters, 0.0);
    for (u32 g = 0; g < groups; g++)
        for (u32 l = 0; l < nl; l++)
            for (u32 t = 0; t < t_total; t++)
                for (u32 f = 0; f < kMaxFilters; f++) {
                    const u32 co = g * kMaxFilters + f;
                    if (co < C_out)
                        wtv[(((size_t)g * nl + l) * t_total + t) * kMaxFilters + f] =
                            wfv[terms[t].w_idx + co * fst + l];
                }
    u32 max_col = 0;
    for (u32 jo = 0; jo < wo; jo++) max_col = std::max(max_col, off[jo + 1] - off[jo]);
    // 21-bit pieces of the weights on the wide limbs
    u64 wide_mask = 0;
    bool wide_ok = nl <= 64, any_wide = false;
    for (u32 l = 0; l < nl; l++) {
        const u64 q = ctx->mod[mod_of(l)];
        any_wide = any_wide || q >= (1ull << 51);
        if (q >= (1ull << 51) && l < 64) wide_mask |= 1ull << l;
        wide_ok = wide_ok && q < (1ull << 63);
    }
    if (!wide_ok) wide_mask = 0;
    const u32 n_wide = (u32)__builtin_popcountll(wide_mask);
    std::vector<double> wpv((size_t)groups * n_wide * t_total * kMaxFilters * kWidePieces, 0.0);
    for (u32 g = 0, wi = 0; g < groups; g++, wi = 0)
        for (u32 l = 0; l < nl; l++) {
            if (!(wide_mask >> l & 1)) continue;
            for (u32 t = 0; t < t_total; t++)
                for (u32 f = 0; f < kMaxFilters; f++) {
                    const u32 co = g * kMaxFilters + f;
                    if (co >= C_out) continue;
                    const u64 v = wv[terms[t].w_idx + co * fst + l];
                    for (u32 j = 0; j < kWidePieces; j++)
                        wpv[((((size_t)g * n_wide + wi) * t_total + t) * kMaxFilters + f) * kWidePieces + j] =
                            (double)((v >> (21 * j)) & ((1ull << 21) - 1));
                }
            wi++;
        }
    wfv.swap(wtv);
    // matrix-core tables: the balanced base-256 digits j of 2^(8a) w mod q
    // for every (filter group, limb, step of 4 terms, tile, lane), one table
    // per distinct sequence of weight rows (interior columns share one)
    bool mfma_ok = ctx->log_n >= 8 && max_col <= kMfmaMaxTerms;
    for (u32 l = 0; l < nl; l++) mfma_ok = mfma_ok && ctx->mod[mod_of(l)] < (1ull << 62);
    std::vector<u64> atv, colv(wo, 0);
    if (mfma_ok) {
        std::map<std::vector<u32>, u64> seen;
        for (u32 jo = 0; jo < wo && mfma_ok; jo++) {
            std::vector<u32> sig;
            for (u32 t = off[jo]; t < off[jo + 1]; t++) sig.push_back(terms[t].w_idx);
            auto it = seen.find(sig);
            if (it != seen.end()) {
                colv[jo] = it->second;
                continue;
            }
            const u32 nt = (u32)sig.size(), steps = (nt + 3) / 4;
            const size_t at0 = atv.size();
            if ((at0 + (size_t)groups * nl * steps * 256) * 8 > (512ull << 20)) {
                mfma_ok = false;
                break;
            }
            atv.resize(at0 + (size_t)groups * nl * steps * 256, 0);
            for (u32 g = 0; g < groups; g++)
                for (u32 l = 0; l < nl; l++) {
                    const u64 q = ctx->mod[mod_of(l)];
                    for (u32 kk = 0; kk < nt; kk++)
                        for (u32 fr = 0; fr < kMaxFilters; fr++) {
                            const u32 co = g * kMaxFilters + fr;
                            if (co >= C_out) continue;
                            const u64 wgt = wv[sig[kk] + co * fst + l];
                            // bytes of w'_a = 2^(8a) w mod q, a = 0..7
                            u64 e[8];
                            for (u32 aa = 0; aa < 8; aa++)
                                e[aa] = balanced_bytes_h((u64)(((u128)wgt << (8 * aa)) % q));
                            const u32 s = kk / 4, lane_hi = kk % 4, h = fr / 4, fi = fr % 4;
                            for (u32 ee = 0; ee < 2; ee++)
                                for (u32 jr = 0; jr < 4; jr++) {
                                    const u32 j = 4 * ee + jr, rho = 4 * fi + jr, T = 2 * h + ee;
                                    u64 word = 0;
                                    for (u32 aa = 0; aa < 8; aa++) word |= ((e[aa] >> (8 * j)) & 0xff) << (8 * aa);
                                    atv[at0 + ((((size_t)g * nl + l) * steps + s) * 4 + T) * 64 + lane_hi * 16 + rho] =
                                        word;
                                }
                        }
                }
            seen[sig] = at0;
            colv[jo] = at0;
        }
    }
    if (!mfma_ok) atv.clear();
    std::vector<u64> kcv;
    if (mfma_ok)
        for (u32 l = 0; l < nl; l++) {
            const u64 q = ctx->mod[mod_of(l)];
            const u64 r64 = (u64)(((u128)1 << 64) % q);
            kcv.push_back((u64)(((u128)1 << 24) % q));
            kcv.push_back((u64)(((u128)1 << 48) % q));
            kcv.push_back((u64)((u128)r64 * r64 % q));
        }
    // one device buffer: terms | off | rot_end | w | ws | bias | wt | wp
    // (8-byte aligned parts)
    size_t b_terms = terms.size() * sizeof(Term), b_off = ((off.size() * 4 + 7) / 8) * 8;
    size_t b_rot = ((rot_end.size() * 4 + 7) / 8) * 8;
    b_off += b_rot;
    const size_t n_words = wv.size() + wsv.size() + bv.size() + wfv.size() + wpv.size();
    size_t total = b_terms + b_off + (n_words + (mfma_ok ? atv.size() + colv.size() + kcv.size() : 0)) * 8;
    auto plan = std::make_shared<ConvPlan>();
    VR_HIP(hipDeviceSynchronize());
    plan->buf = dev_alloc(ctx, total, nullptr);
    char* base = (char*)plan->buf->ptr;
    std::vector<char> h(total, 0);
    memcpy(h.data(), terms.data(), b_terms);
    memcpy(h.data() + b_terms, off.data(), off.size() * 4);
    memcpy(h.data() + b_terms + (b_off - b_rot), rot_end.data(), rot_end.size() * 4);
    size_t o = b_terms + b_off;
    memcpy(h.data() + o, wv.data(), wv.size() * 8);
    memcpy(h.data() + o + wv.size() * 8, wsv.data(), wsv.size() * 8);
    memcpy(h.data() + o + (wv.size() + wsv.size()) * 8, bv.data(), bv.size() * 8);
    memcpy(h.data() + o + (wv.size() + wsv.size() + bv.size()) * 8, wfv.data(), wfv.size() * 8);
    memcpy(h.data() + o + (wv.size() + wsv.size() + bv.size() + wfv.size()) * 8, wpv.data(), wpv.size() * 8);
    if (mfma_ok) {
        memcpy(h.data() + o + n_words * 8, atv.data(), atv.size() * 8);
        memcpy(h.data() + o + (n_words + atv.size()) * 8, colv.data(), colv.size() * 8);
        memcpy(h.data() + o + (n_words + atv.size() + colv.size()) * 8, kcv.data(), kcv.size() * 8);
    }
    VR_HIP(hipMemcpy(base, h.data(), total, hipMemcpyHostToDevice));
    plan->terms = (const Term*)base;
    plan->off = (const u32*)(base + b_terms);
    plan->rot_end = (const u32*)(base + b_terms + (b_off - b_rot));
    plan->w = (const u64*)(base + o);
    plan->ws = plan->w + wv.size();
    plan->bias = plan->ws + wsv.size();
    plan->wt = (const double*)(plan->bias + bv.size());
    plan->wp = plan->wt + wfv.size();
    plan->wide_mask = wide_mask;
    plan->n_wide = n_wide;
    plan->any_wide = any_wide;
    if (mfma_ok) {
        plan->at = plan->w + n_words;
        plan->col_at = plan->at + atv.size();
        plan->kc = plan->col_at + colv.size();
    }
    plan->t_total = t_total;
    plan->max_col = max_col;
    ctx->plans[key] = plan;
    return *plan;
}

}  // namespace

Slab layer_square(vr_context* ctx, const vr_eval_keys* ek, const Slab& in, hipStream_t s)
{
    return square_slab(ctx, ek, in, s);
}

Slab fc_slab(vr_context* ctx, const vr_eval_keys* ek, const Slab& y, const u64* P, u64 p_stride,
             double p_scale, u32 p_level, u32 n_out, const double* bias, u32 block, hipStream_t s, u32 p_rep)
{
    if (y.ncomp != 2) throw Error(VR_EINVAL, "FC inputs must be 2-component");
    // weights encoded below the inputs' level: the inputs are read on limbs
    // 0..p_level only (a level drop keeps the message), so the products, the
    // rescale and the rotate-and-sum all run at the weights' level
    const u32 level = std::min(y.level, p_level);
    if (level < 1) throw Error(VR_ELEVEL, "FC needs a level to rescale");
    const u32 nl = level + 1;
    Slab acc = new_slab(ctx, n_out, 2, level, y.scale * p_scale, s);
    dim3 grid((ctx->n + kThreads - 1) / kThreads, nl, (n_out + kFcGroup - 1) / kFcGroup);
    hipLaunchKernelGGL(k_mulplain_acc, grid, dim3(kThreads), 0, s, acc.base, acc.stride, y.base,
                       y.stride, (u64)(y.level + 1) * ctx->n, y.n, P, p_stride, n_out, nl, ctx->log_n,
                       ctx->d_modq, p_rep);
    VR_CHECK_LAUNCH();
    Slab z = rescale_slab(ctx, acc, s);
    // rotate-and-sum inside each block: z += Rot(z, 2^t)
    for (u32 st = 1; st < block; st <<= 1) {
        std::vector<Slab> r;
        rotate_slab(ctx, ek, z, {(int32_t)st}, r, s);
        launch_addsub(ctx, z.base, z.base, r[0].base, z.n * 2, z.level + 1, false, s);
    }
    // bias on the constant coefficient of c0 (every evaluation slot)
    for (u32 o = 0; o < n_out; o++) {
        LimbConsts kc;
        for (u32 l = 0; l <= z.level; l++) kc.c[l] = double_to_mod(bias[o] * z.scale, ctx->mod[l]);
        launch_add_scalar(ctx, z.ct(o), z.ct(o), z.level + 1, kc, s);
    }
    return z;
}

// Weight plaintexts as one [n_out * n_in][>= nl][N] array: in place when the
// handles already form one (as vr_encode_fc_weights returns them), else a copy.
const u64* fc_weights(vr_context* ctx, const vr_plaintext* const* W_pt, size_t count, u32 nl,
                      u64* p_stride, double* p_scale, u32* p_level, BufPtr& holder, hipStream_t s,
                      u32* p_rep)
{
    const vr_plaintext* p0 = W_pt[0];
    if (!p0) throw Error(VR_EINVAL, "null plaintext");
    const u64 stride = (u64)(p0->level + 1) * ctx->n;
    bool contiguous = true;
    // the compact copies (runs of 2^clog equal words kept once), when every
    // plaintext has one with the same run length, laid out back to back
    bool compact = p0->cdata != nullptr && p0->clog > 0;
    const u64 cstride = compact ? (u64)(p0->level + 1) * (ctx->n >> p0->clog) : 0;
    for (size_t i = 0; i < count; i++) {
        if (!W_pt[i]) throw Error(VR_EINVAL, "null plaintext");
        if (W_pt[i]->level != p0->level) throw Error(VR_ELEVEL, "weight plaintexts at different levels");
        if (W_pt[i]->scale != p0->scale) throw Error(VR_ESCALE, "weight plaintexts at different scales");
        contiguous = contiguous && W_pt[i]->data == p0->data + i * stride;
        compact = compact && W_pt[i]->clog == p0->clog && W_pt[i]->cdata == p0->cdata + i * cstride;
    }
    if (knob(ctx, "fc_compact") == 1) compact = false;
    *p_scale = p0->scale;
    // the layer runs at min(input level, weight level): nl limbs are read
    nl = std::min(nl, p0->level + 1);
    *p_level = nl - 1;
    *p_rep = 0;
    if (compact) {
        *p_stride = cstride;
        *p_rep = p0->clog;
        return p0->cdata;
    }
    if (contiguous) {
        *p_stride = stride;
        return p0->data;
    }
    const u64 ws = (u64)nl * ctx->n;
    holder = dev_alloc(ctx, count * ws * sizeof(u64), s);
    for (size_t i = 0; i < count; i++)
        VR_HIP(hipMemcpyAsync(as_u64(holder) + i * ws, W_pt[i]->data, ws * sizeof(u64),
                              hipMemcpyDeviceToDevice, s));
    *p_stride = ws;
    return as_u64(holder);
}

// ------------------------------------------------------------- encodings

vr_ciphertext** encrypt_slots_batch(vr_context* ctx, const vr_eval_keys* ek,
                                    const std::vector<double>& slots, u32 n_ct, u32 level,
                                    const Seed256& seed, u64 first_id, vr_ciphertext** out, hipStream_t s)
{
    // encode every vector in one batched FFT, then encrypt each into one slab
    const size_t n = ctx->n, S = ctx->slots;
    const u32 nl = level + 1;
    BufPtr xd = dev_alloc(ctx, slots.size() * sizeof(double), s);
    VR_HIP(hipMemcpyAsync(xd->ptr, slots.data(), slots.size() * sizeof(double), hipMemcpyHostToDevice, s));
    BufPtr mb = dev_alloc(ctx, (size_t)n_ct * nl * n * sizeof(u64), s);
    encode_to_limbs(ctx, (const double*)xd->ptr, (u32)S, n_ct, S, ctx->scale, as_u64(mb), nl,
                    (u64)nl * n, s);
    ntt_forward(ctx, poly_limbs(as_u64(mb), as_u64(mb), n_ct, nl, (u64)nl * n, (int)level), s);
    Slab sl = new_slab(ctx, n_ct, 2, level, ctx->scale, s);
    BufPtr ints = dev_alloc(ctx, 3 * n * sizeof(i64), s);
    BufPtr limbs = dev_alloc(ctx, (size_t)3 * nl * n * sizeof(u64), s);
    i64* vi = (i64*)ints->ptr;
    u64* L3 = as_u64(limbs);
    std::vector<u32> mods(nl);
    for (u32 l = 0; l < nl; l++) mods[l] = l;
    for (u32 c = 0; c < n_ct; c++) {
        u64 id = first_id + c;
        launch_sample_ternary(ctx, vi, seed, kPurEncV, id, s);
        launch_sample_gauss(ctx, vi + n, seed, kPurEncE0, id, s);
        launch_sample_gauss(ctx, vi + 2 * n, seed, kPurEncE1, id, s);
        for (int k = 0; k < 3; k++) launch_int_to_limbs(ctx, L3 + (size_t)k * nl * n, vi + k * n, mods.data(), nl, s);
        ntt_forward(ctx, poly_limbs(L3, L3, 3, nl, (u64)nl * n, (int)level), s);
        launch_encrypt_combine(ctx, sl.ct(c), L3, L3 + (size_t)nl * n, L3 + (size_t)2 * nl * n,
                               ek->pk, as_u64(mb) + (size_t)c * nl * n, nl, s);
    }
    to_handles(ctx, sl, out);
    return out;
}

// The conv's rotations and linear combination over `keys` (ciphertexts of x
// in the ranges of each session), one network per call of conv_lincomb_into.
// Lazy form when the kernel rotates (k > 1) and the special primes are no
// more than the Q limbs (K <= level + 1, so the extended basis at most doubles
// the limbs): the rotations by 1..k-1 of every column stay in the extended
// basis (no ModDown), the sums are taken there, and one ModDown by P q_l per
// output both finishes the key switches and rescales.  Otherwise the plain
// form: rotations with their ModDown, sums in Q, a rescale.
struct ConvRot {
    std::vector<Slab> rot;
    bool ext = false;
    u32 keep = 0;
};

bool conv_lazy(vr_context* ctx, u32 k, u32 level) { return k > 1 && ctx->K <= level + 1; }

// keep > 0 (lazy form only): the sums and the ModDown make output limbs
// q_0..q_{keep-1} alone (a consumer that reads no others)
ConvRot conv_rotations(vr_context* ctx, const std::vector<KeyRange>& keys, const Slab& x, u32 k, hipStream_t s,
                       u32 keep)
{
    ConvRot cr;
    std::vector<int32_t> steps;
    for (u32 u = 1; u < k; u++) steps.push_back((int32_t)u);
    if (steps.empty()) return cr;
    cr.ext = conv_lazy(ctx, k, x.level);
    cr.keep = cr.ext ? keep : 0;
    if (cr.ext)
        rotate_slab_ext(ctx, keys, x, steps, cr.rot, s, cr.keep);
    else
        rotate_slab_keyed(ctx, keys, x, steps, cr.rot, s);
    return cr;
}

// out (n_sets * C_out * w_out ciphertexts, extended when cr.ext) = the
// linear combination of the inputs x_in (n_sets sets of C_in * w columns)
// and their rotations cr.rot[u - 1] starting at ciphertext r_at
void conv_lincomb_into(vr_context* ctx, const Slab& out, u32 out_at, const Slab& x, u32 x_at, const ConvRot& cr,
                       u32 r_at, u32 n_sets, u32 C_in, u32 w, u32 pad, const double* K, const double* bias,
                       u32 C_out, u32 k, u32 stride, hipStream_t s)
{
    const u32 level = x.level, nq = level + 1;
    const u32 wo = (w + 2 * pad - k) / stride + 1, n_out = C_out * wo;
    const double out_scale = x.scale * (double)ctx->mod[level];
    const ConvPlan& plan = conv_plan(ctx, C_in, w, pad, K, bias, C_out, k, stride, level, out_scale, cr.ext,
                                     cr.keep);
    const u32 nk = cr.keep ? cr.keep : level;
    const u32 nl = cr.ext ? nk + 1 + ctx->K : nq;
    const Slab& r = cr.rot.empty() ? x : cr.rot[0];
    // cpb 256-coefficient chunks per block share one copy of its weights
    const u32 chunks = (ctx->n + kThreads - 1) / kThreads;
    const u32 cpb = chunks >= 16 ? 4 : 1;
    const u32 total = ((chunks + cpb - 1) / cpb) * 2 * nl * n_sets * wo;
    const u32 per_xcd = (total + 7) / 8;
    const size_t shmem = (size_t)std::min(plan.max_col, kTermChunk) * kMaxFilters * sizeof(double);
    // rows on moduli of 2^51 or more by k_lincomb_wide unless the knob
    // lincomb_wide is off (or the pieces do not apply): k_lincomb's integer
    // products then
    const bool wide = plan.n_wide > 0 && knob(ctx, "lincomb_wide") == 0;
    ProfScope prof(ctx, kProfLincomb, s, (u64)n_sets * n_out * 2 * nl);
    if (plan.at && knob(ctx, "lincomb_mfma") == 0) {
        for (int fp = 1; fp >= 0; fp--) {
            if (!fp && !plan.any_wide) break;
            hipLaunchKernelGGL(fp ? k_lincomb_mfma<true> : k_lincomb_mfma<false>, dim3(8 * per_xcd), dim3(kThreads),
                               0, s, out.ct(out_at), out.stride, x.ct(x_at), cr.rot.empty() ? x.ct(x_at) : r.ct(r_at),
                               C_in * w, n_sets, x.stride, r.stride, (u64)r.n * r.stride, plan.terms, plan.off,
                               plan.rot_end, plan.at, plan.col_at, plan.kc, plan.bias, nl, nk, level, ctx->L - nk, nq,
                               ctx->log_n, ctx->d_modq, wo, C_out, total, per_xcd, cpb);
            VR_CHECK_LAUNCH();
        }
        return;
    }
    for (int fp = 1; fp >= 0; fp--) {
        if (!fp && (wide || !plan.any_wide)) break;
        hipLaunchKernelGGL(fp ? k_lincomb<true> : k_lincomb<false>, dim3(8 * per_xcd), dim3(kThreads),
                           fp ? shmem : 0, s, out.ct(out_at), out.stride, x.ct(x_at),
                           cr.rot.empty() ? x.ct(x_at) : r.ct(r_at), C_in * w, n_sets, x.stride, r.stride,
                           (u64)r.n * r.stride, plan.terms, plan.off, plan.rot_end, plan.w, plan.ws, plan.wt,
                           plan.t_total, C_in * k * k, plan.bias, nl, nk, level, ctx->L - nk, nq, ctx->log_n,
                           ctx->d_modq, wo, C_out, total, per_xcd, cpb);
        VR_CHECK_LAUNCH();
    }
    if (wide) {
        const u32 wtotal = ((chunks + cpb - 1) / cpb) * 2 * plan.n_wide * n_sets * wo;
        const u32 wper = (wtotal + 7) / 8;
        const size_t wsh = (size_t)std::min(plan.max_col, kWideChunk) * kMaxFilters * kWidePieces * sizeof(double);
        hipLaunchKernelGGL(k_lincomb_wide, dim3(8 * wper), dim3(kThreads), wsh, s, out.ct(out_at), out.stride,
                           x.ct(x_at), cr.rot.empty() ? x.ct(x_at) : r.ct(r_at), C_in * w, n_sets, x.stride,
                           r.stride, (u64)r.n * r.stride, plan.terms, plan.off, plan.rot_end, plan.wp, plan.t_total,
                           plan.bias, nl, nk, level, ctx->L - nk, nq, ctx->log_n, ctx->d_modq, wo, C_out,
                           plan.wide_mask, plan.n_wide, wtotal, wper, cpb);
        VR_CHECK_LAUNCH();
    }
}

// Conv layer over n_sets image sets laid out in one slab (set s occupies
// ciphertexts s * C_in * w .. (s + 1) * C_in * w - 1): one hoisted ModUp per
// column, one shared-key inner-product launch per rotation step for every
// column of every set (rotations kept in the extended basis), one fused
// MulConst/AddConst launch, one ModDown by P q_l per output.
Slab conv_slab(vr_context* ctx, const vr_eval_keys* ek, const Slab& x, u32 n_sets, u32 C_in, u32 w,
               u32 pad, const double* K, const double* bias, u32 C_out, u32 k, u32 stride,
               hipStream_t s)
{
    if (x.ncomp != 2 || x.ext) throw Error(VR_EINVAL, "conv inputs must be 2-component");
    if (x.level < 1) throw Error(VR_ELEVEL, "conv needs a level to rescale");
    const u32 wo = (w + 2 * pad - k) / stride + 1;
    const u32 level = x.level;
    ConvRot cr = conv_rotations(ctx, {KeyRange{0, x.n, ek}}, x, k, s, 0);
    const double out_scale = x.scale * (double)ctx->mod[level];
    const u32 n_out = C_out * wo;
    Slab acc = cr.ext ? new_ext_slab(ctx, n_sets * n_out, level, out_scale, s)
                      : new_slab(ctx, n_sets * n_out, 2, level, out_scale, s);
    conv_lincomb_into(ctx, acc, 0, x, 0, cr, 0, n_sets, C_in, w, pad, K, bias, C_out, k, stride, s);
    cr.rot.clear();
    return cr.ext ? mod_down_rescale_slab(ctx, acc, s) : rescale_slab(ctx, acc, s);
}

// Several column-split products at one level and scale in one schedule
// (S-MM of the abstract and "Homomorphic Matrix Multiplication" per request):
// the Bbar columns of every request share one hoisted ModUp; requests are
// ordered by P' (largest first) so that for each rotation step idx the
// ciphertexts still needing it form a prefix, rotated by one shared-key
// inner product and one ModDown; the tensor accumulations stay per request,
// and every request's P' products are relinearised and rescaled together.
std::vector<Slab> matmul_multi(vr_context* ctx, const vr_eval_keys* ek, const std::vector<MatReq>& reqs_in,
                               hipStream_t s)
{
    const u32 nr = (u32)reqs_in.size();
    if (nr == 0) return {};
    // m < p: the transposed product C^T = B^T A^T on the same ciphertexts
    // with their roles swapped (the Bbar columns are the A-role columns of
    // B^T, the A columns the Bbar-role columns of A^T)
    std::vector<MatReq> reqs = reqs_in;
    for (MatReq& q : reqs)
        if (q.m < q.p) std::swap(q.A, q.B), std::swap(q.m, q.p);
    const u32 level = reqs[0].A.level, nl = level + 1;
    const double scale_ab = reqs[0].A.scale * reqs[0].B.scale;
    std::vector<u32> order(nr), Pp(nr);
    for (u32 r = 0; r < nr; r++) {
        const MatReq& q = reqs[r];
        if (q.A.level != level || q.B.level != level) throw Error(VR_ELEVEL, "matmul inputs at different levels");
        if (q.A.scale * q.B.scale != scale_ab) throw Error(VR_ESCALE, "matmul inputs at different scales");
        if (q.A.ncomp != 2 || q.B.ncomp != 2) throw Error(VR_EINVAL, "matmul inputs must be 2-component");
        Pp[r] = pow2ceil(q.p);
        order[r] = r;
        for (u32 i = 1; i < Pp[r]; i++) (void)rot_key(ek, galois_element(ctx, (int32_t)i));
    }
    std::stable_sort(order.begin(), order.end(), [&](u32 a, u32 b) { return Pp[a] > Pp[b]; });
    const size_t N = ctx->n;
    // every request's Bbar columns in one slab, in that order; products slab
    u32 n_tot = 0, p_tot = 0;
    std::vector<u32> b_off(nr), t_off(nr);
    for (u32 r : order) b_off[r] = n_tot, n_tot += reqs[r].n;
    for (u32 r = 0; r < nr; r++) t_off[r] = p_tot, p_tot += Pp[r];
    Slab SB = reqs[0].B;   // one request: its Bbar columns in place
    if (nr > 1) {
        SB = new_slab(ctx, n_tot, 2, level, reqs[0].B.scale, s);
        for (u32 r = 0; r < nr; r++)
            VR_HIP(hipMemcpyAsync(SB.ct(b_off[r]), reqs[r].B.base, (size_t)reqs[r].n * SB.stride * sizeof(u64),
                                  hipMemcpyDeviceToDevice, s));
    }
    Slab T = new_slab(ctx, p_tot, 3, level, scale_ab, s);
    dim3 grid((ctx->n + kThreads - 1) / kThreads, nl);
    for (u32 r = 0; r < nr; r++) {   // idx = 0: no rotation
        hipLaunchKernelGGL(k_tensor_acc, grid, dim3(kThreads), 0, s, T.ct(t_off[r]), reqs[r].A.base,
                           reqs[r].A.stride, SB.ct(b_off[r]), SB.stride, reqs[r].n, nl, ctx->log_n,
                           ctx->d_modq, 0u);
        VR_CHECK_LAUNCH();
    }
    const u32 max_p = Pp[order[0]];
    if (max_p > 1) {
        // Bbar columns in chunks whose key-switch scratch stays bounded: one
        // hoisted ModUp per chunk, then every rotation step its columns need;
        // a request's tensor sum over k is accumulated chunk by chunk (the
        // chunk holding its first column starts it).
        KsShape k = ks_shape(ctx, level);
        const u64 xs = (u64)k.beta * k.next * N, us = (u64)2 * k.next * N;
        const u32 cs = switch_chunk(ctx, level, n_tot);
        BufPtr xbuf = dev_alloc(ctx, ((size_t)cs * xs + (size_t)cs * k.nq * N) * sizeof(u64), s);
        u64* X = as_u64(xbuf);
        BufPtr ubuf = dev_alloc(ctx, ((size_t)cs * us + keyswitch_moddown_scratch(ctx, level, cs)) * sizeof(u64), s);
        u64* U = as_u64(ubuf);
        Slab R = new_slab(ctx, cs, 2, level, SB.scale, s);
        for (u32 c0 = 0; c0 < n_tot; c0 += cs) {
            const u32 nc = std::min(cs, n_tot - c0);
            keyswitch_modup_batch(ctx, SB.ct(c0) + (size_t)k.nq * N, SB.stride, nc, level, X,
                                  X + (size_t)cs * xs, s);
            for (u32 idx = 1; idx < max_p; idx++) {
                u32 n_act = 0;   // prefix of columns whose request still needs step idx
                for (u32 r : order)
                    if (Pp[r] > idx) n_act = b_off[r] + reqs[r].n;
                if (n_act <= c0) break;   // the prefix only shrinks as idx grows
                const u32 na = std::min(nc, n_act - c0);
                const u32 g = galois_element(ctx, (int32_t)idx);
                keyswitch_inner_batch(ctx, X, xs, SB.ct(c0) + (size_t)k.nq * N, SB.stride, na,
                                      rot_key(ek, g).data, level, g, U, us, s);
                keyswitch_moddown_batch(ctx, U, us, na, level, R.base, R.base + (size_t)k.nq * N, R.stride,
                                        SB.ct(c0), g, nullptr, SB.stride, U + (size_t)na * us, s);
                for (u32 r : order) {
                    if (Pp[r] <= idx) continue;
                    // columns [k0, k1) of request r inside this chunk
                    const u32 lo = std::max(b_off[r], c0), hi = std::min(b_off[r] + reqs[r].n, c0 + na);
                    if (lo >= hi) continue;
                    const u32 k0 = lo - b_off[r];
                    hipLaunchKernelGGL(k_tensor_acc, grid, dim3(kThreads), 0, s, T.ct(t_off[r] + idx),
                                       reqs[r].A.ct(k0), reqs[r].A.stride, R.ct(lo - c0), R.stride, hi - lo,
                                       nl, ctx->log_n, ctx->d_modq, k0 > 0 ? 1u : 0u);
                    VR_CHECK_LAUNCH();
                }
            }
        }
    }
    Slab out = relin_rescale_slab(ctx, ek, T, s);
    std::vector<Slab> res(nr);
    for (u32 r = 0; r < nr; r++) {
        res[r] = out;
        res[r].n = Pp[r];
        res[r].base = out.ct(t_off[r]);
    }
    return res;
}

// Outer-product products (the rotation-free form of the split product) of
// several requests at one level and scale: row tile t of request r
// accumulates sum_k Tensor(A'_{t,k}, B'_k) (A' tile-major, t n + k), then
// every tile of every request is relinearised and rescaled together.  No
// rotation.
std::vector<Slab> matmul_outer_multi(vr_context* ctx, const vr_eval_keys* ek, const std::vector<MatReq>& reqs,
                                     hipStream_t s)
{
    const u32 nr = (u32)reqs.size();
    if (nr == 0) return {};
    const u32 level = reqs[0].A.level, nl = level + 1;
    const double scale_ab = reqs[0].A.scale * reqs[0].B.scale;
    std::vector<u32> T(nr), off(nr);
    u32 tiles = 0;
    for (u32 r = 0; r < nr; r++) {
        const MatReq& q = reqs[r];
        if (q.A.level != level || q.B.level != level) throw Error(VR_ELEVEL, "matmul inputs at different levels");
        if (q.A.scale * q.B.scale != scale_ab) throw Error(VR_ESCALE, "matmul inputs at different scales");
        if (q.A.ncomp != 2 || q.B.ncomp != 2) throw Error(VR_EINVAL, "matmul inputs must be 2-component");
        u32 Pp, R;
        outer_tiles(ctx, q.m, q.p, &Pp, &R, &T[r]);
        if (q.A.n != T[r] * q.n || q.B.n != q.n) throw Error(VR_EINVAL, "outer product needs T n and n ciphertexts");
        off[r] = tiles;
        tiles += T[r];
    }
    Slab acc = new_slab(ctx, tiles, 3, level, scale_ab, s);
    dim3 grid((ctx->n + kThreads - 1) / kThreads, nl);
    for (u32 r = 0; r < nr; r++)
        for (u32 t = 0; t < T[r]; t++) {
            hipLaunchKernelGGL(k_tensor_acc, grid, dim3(kThreads), 0, s, acc.ct(off[r] + t), reqs[r].A.ct(t * reqs[r].n),
                               reqs[r].A.stride, reqs[r].B.base, reqs[r].B.stride, reqs[r].n, nl, ctx->log_n,
                               ctx->d_modq, 0u);
            VR_CHECK_LAUNCH();
        }
    Slab out = relin_rescale_slab(ctx, ek, acc, s);
    std::vector<Slab> res(nr);
    for (u32 r = 0; r < nr; r++) {
        res[r] = out;
        res[r].n = T[r];
        res[r].base = out.ct(off[r]);
    }
    return res;
}

// (P', Mb, c, nb) of the column-block form: blocks of Mb = P' ceil((m + P' -
// 1) / P') slots, c (a power of two, c Mb <= S, c <= pow2(n)) columns per
// ciphertext, nb = ceil(n / c) ciphertexts per operand
void block_shape(vr_context* ctx, u32 m, u32 n, u32 p, u32* Pp, u32* Mb, u32* c, u32* nb)
{
    *Pp = pow2ceil(p);
    const u64 mb = (u64)*Pp * (((u64)m + *Pp - 1 + *Pp - 1) / *Pp);
    if (mb > ctx->slots) throw Error(VR_EINVAL, "m + P' - 1 exceeds the slot count");
    *Mb = (u32)mb;
    u32 cc = 1;
    while ((u64)2 * cc * mb <= ctx->slots && cc < pow2ceil(n)) cc *= 2;
    *c = cc;
    *nb = (n + cc - 1) / cc;
}

// (P', R, T) of the outer-product form: column padding, rows per ciphertext,
// row tiles
void outer_tiles(vr_context* ctx, u32 m, u32 p, u32* Pp, u32* R, u32* T)
{
    *Pp = pow2ceil(p);
    if (*Pp > ctx->slots) throw Error(VR_EINVAL, "p exceeds the slot count");
    *R = (u32)(ctx->slots / *Pp);
    *T = (m + *R - 1) / *R;
}

// x^2 followed by the FC with one relinearisation per FC output (lazy
// relinearisation) when the FC level l >= 2 leaves room for the tensors'
// weight products: with e the binary exponent of y_scale^2 p_scale (the
// product scale is below 2^e) and b the total bit length of q_0..q_l,
// e + l + 12 <= b keeps 2^10 times the scale below Q_l / 2.
bool square_fc_lazy(vr_context* ctx, double y_scale, double p_scale, u32 fl)
{
    if (fl < 2) return false;
    int e = 0;
    (void)std::frexp(y_scale * y_scale * p_scale, &e);
    int bits = 0;
    for (u32 i = 0; i <= fl; i++) bits += 64 - __builtin_clzll(ctx->mod[i]);
    return e + (int)fl + 12 <= bits;
}

Slab run_cnn_multi(vr_context* ctx, const std::vector<NetSeg>& segs, const Slab& x, hipStream_t s)
{
    if (segs.empty()) throw Error(VR_EINVAL, "empty wave");
    const CnnDesc& d0 = *segs[0].d;
    u32 n_in = 0;
    for (const NetSeg& g : segs) {
        const CnnDesc& d = *g.d;
        if (d.k != d0.k || d.square != d0.square || (d.fc_out != 0) != (d0.fc_out != 0) ||
            (d.fc_out && (d.fc_level != d0.fc_level || d.fc_scale != d0.fc_scale)))
            throw Error(VR_EINVAL, "wave segments must share kernel size, x^2, FC presence and FC level");
        n_in += g.n_sets * d.n_in();
    }
    if (x.n != n_in || x.ncomp != 2) throw Error(VR_EINVAL, "wave input slab does not match its segments");
    if (x.level < 1) throw Error(VR_ELEVEL, "conv needs a level to rescale");
    const u32 level = x.level;
    // conv: rotations of every input column by 1..k-1 under each session's keys
    std::vector<KeyRange> kin;
    u32 at = 0;
    for (const NetSeg& g : segs) {
        kin.push_back(KeyRange{at, at + g.n_sets * g.d->n_in(), g.ek});
        at = kin.back().end;
    }
    const double out_scale = x.scale * (double)ctx->mod[level];
    // x^2 and FC fused: the squares' tensors meet the FC weights
    // unrelinearised, on the FC level's limbs only; the conv then makes just
    // those limbs of its outputs (they are all the FC reads)
    const double y_scale = out_scale / (double)ctx->mod[level];
    const u32 fl0 = std::min(level - 1, d0.fc_level);
    const bool lazy_fc = d0.square && d0.fc_out && square_fc_lazy(ctx, y_scale, d0.fc_scale, fl0);
    const bool prune = knob(ctx, "conv_prune") == 0;
    const u32 keep = lazy_fc && prune && fl0 + 1 < level ? fl0 + 1 : 0;
    ConvRot cr = conv_rotations(ctx, kin, x, d0.k, s, keep);
    u32 n_conv = 0;
    for (const NetSeg& g : segs) n_conv += g.n_sets * g.d->C_out * g.d->w_out();
    Slab acc = cr.ext ? new_ext_slab(ctx, n_conv, level, out_scale, s, cr.keep)
                      : new_slab(ctx, n_conv, 2, level, out_scale, s);
    // the linear combination per network, on its own inputs and rotations
    std::vector<KeyRange> kout;
    u32 in_at = 0, out_at = 0;
    for (const NetSeg& g : segs) {
        const CnnDesc& d = *g.d;
        const u32 n_out = d.C_out * d.w_out();
        conv_lincomb_into(ctx, acc, out_at, x, in_at, cr, in_at, g.n_sets, d.C_in, d.w, d.pad, d.K.data(),
                          d.bias.data(), d.C_out, d.k, d.stride, s);
        kout.push_back(KeyRange{out_at, out_at + g.n_sets * n_out, g.ek});
        in_at += g.n_sets * d.n_in();
        out_at += g.n_sets * n_out;
    }
    cr.rot.clear();
    Slab y = cr.ext ? mod_down_rescale_slab(ctx, acc, s) : rescale_slab(ctx, acc, s);
    acc = Slab();
    if (y.scale != y_scale) throw Error(VR_EINVAL, "conv output scale differs from its prediction");
    if (cr.keep && y.level != fl0) throw Error(VR_EINVAL, "pruned conv output at the wrong level");
    if (d0.square && !lazy_fc) {
        // tensor of everything, relinearisation per session, one rescale
        Slab T = new_slab(ctx, y.n, 3, y.level, y.scale * y.scale, s);
        dim3 grid((ctx->n + kThreads - 1) / kThreads, y.n * (y.level + 1));
        {
            ProfScope prof(ctx, kProfTensor, s, (u64)y.n * 2 * (y.level + 1));
            hipLaunchKernelGGL(k_tensor_batch, grid, dim3(kThreads), 0, s, T.base, y.base, y.base, y.stride,
                               y.level + 1, ctx->log_n, ctx->d_modq);
            VR_CHECK_LAUNCH();
        }
        y = relin_slab_keyed(ctx, kout, T, s, true);
    }
    if (!d0.fc_out) return y;
    // FC: weight products per network and set at the weights' level, one
    // rescale (lazy: the relinearisation fused with a rescale, then a second
    // rescale), the rotate-and-sum over each set's block (segments in
    // decreasing block order, so the ones still summing form a prefix)
    const u32 fl = std::min(y.level, d0.fc_level);
    if (fl < 1) throw Error(VR_ELEVEL, "FC needs a level to rescale");
    u32 n_fc = 0;
    for (size_t i = 0; i < segs.size(); i++) {
        n_fc += segs[i].n_sets * segs[i].d->fc_out;
        if (i && segs[i].d->fc_block > segs[i - 1].d->fc_block)
            throw Error(VR_EINVAL, "FC segments must come in decreasing block order");
    }
    Slab z = lazy_fc ? new_slab(ctx, n_fc, 3, fl, y.scale * y.scale * d0.fc_scale, s)
                     : new_slab(ctx, n_fc, 2, fl, y.scale * d0.fc_scale, s);
    std::vector<KeyRange> kfc;
    u32 y_at = 0, z_at = 0;
    for (const NetSeg& g : segs) {
        const CnnDesc& d = *g.d;
        const u32 per = d.C_out * d.w_out();
        for (u32 st = 0; st < g.n_sets; st++) {
            dim3 grid((ctx->n + kThreads - 1) / kThreads, fl + 1, (d.fc_out + kFcGroup - 1) / kFcGroup);
            ProfScope prof(ctx, kProfTensor, s, (u64)d.fc_out * (lazy_fc ? 3 : 2) * (fl + 1));
            if (lazy_fc) {
                // FP64 rows, then the rows of 2^51 or more
                const dim3 sg(ctx->n / 64, fl + 1, (d.fc_out + kSqfcGroup - 1) / kSqfcGroup);
                for (int fp = 1; fp >= 0; fp--) {
                    hipLaunchKernelGGL(fp ? k_sqfc_acc<true> : k_sqfc_acc<false>, sg, dim3(kThreads), 0, s,
                                       z.ct(z_at + st * d.fc_out), z.stride, y.ct(y_at + st * per), y.stride,
                                       (u64)(y.level + 1) * ctx->n, per, d.fc_P, d.fc_stride, d.fc_out, fl + 1,
                                       ctx->log_n, ctx->d_modq, d.fc_rep);
                    VR_CHECK_LAUNCH();
                }
            } else
                hipLaunchKernelGGL(k_mulplain_acc, grid, dim3(kThreads), 0, s, z.ct(z_at + st * d.fc_out), z.stride,
                                   y.ct(y_at + st * per), y.stride, (u64)(y.level + 1) * ctx->n, per, d.fc_P,
                                   d.fc_stride, d.fc_out, fl + 1, ctx->log_n, ctx->d_modq, d.fc_rep);
            VR_CHECK_LAUNCH();
        }
        kfc.push_back(KeyRange{z_at, z_at + g.n_sets * d.fc_out, g.ek});
        y_at += g.n_sets * per;
        z_at += g.n_sets * d.fc_out;
    }
    y = Slab();
    if (lazy_fc) z = relin_slab_keyed(ctx, kfc, z, s, true);
    z = rescale_slab(ctx, z, s);
    for (u32 step = 1; step < segs[0].d->fc_block; step <<= 1) {
        std::vector<KeyRange> act;
        for (size_t i = 0; i < segs.size(); i++)
            if (segs[i].d->fc_block > step) act.push_back(kfc[i]);
        Slab za = z;
        za.n = act.back().end;
        std::vector<Slab> r;
        rotate_slab_keyed(ctx, act, za, {(int32_t)step}, r, s);
        launch_addsub(ctx, za.base, za.base, r[0].base, za.n * 2, za.level + 1, false, s);
    }
    z_at = 0;
    for (const NetSeg& g : segs) {
        for (u32 st = 0; st < g.n_sets; st++)
            for (u32 o = 0; o < g.d->fc_out; o++) {
                LimbConsts kc;
                for (u32 l = 0; l <= z.level; l++) kc.c[l] = double_to_mod(g.d->fc_bias[o] * z.scale, ctx->mod[l]);
                launch_add_scalar(ctx, z.ct(z_at + st * g.d->fc_out + o), z.ct(z_at + st * g.d->fc_out + o),
                                  z.level + 1, kc, s);
            }
        z_at += g.n_sets * g.d->fc_out;
    }
    return z;
}

}  // namespace vr

using namespace vr;

#define API_BEGIN try {
#define API_END                                                  \
    }                                                            \
    catch (const vr::Error& e)                                   \
    {                                                            \
        set_last_error(e.what());                                \
        return e.code;                                           \
    }                                                            \
    catch (const std::bad_alloc&)                                \
    {                                                            \
        set_last_error("host allocation failed");                \
        return VR_ENOMEM;                                        \
    }                                                            \
    catch (const std::exception& e)                              \
    {                                                            \
        set_last_error(e.what());                                \
        return VR_EINVAL;                                        \
    }                                                            \
    return VR_OK;

#define REQUIRE(cond, msg) \
    if (!(cond)) throw Error(VR_EINVAL, msg)

extern "C" {

vr_status vr_encrypt_columns(vr_context* ctx, const vr_eval_keys* ek, const double* x, uint32_t B,
                             uint32_t C, uint32_t h, uint32_t w, uint32_t pad, uint32_t level,
                             const uint64_t* seed, uint64_t first_ct_id, vr_ciphertext** cols)
{
    if (cols)
        for (size_t i = 0; i < (size_t)C * w; i++) cols[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && x && cols && seed, "null argument");
    REQUIRE(B >= 1 && C >= 1 && h >= 1 && w >= 1, "empty image batch");
    REQUIRE(level <= ctx->L, "level above the modulus chain");
    const u32 Hp = pow2ceil(h + 2 * pad);
    REQUIRE((size_t)B * Hp <= ctx->slots, "B * pow2(h + 2 pad) exceeds the slot count");
    const size_t S = ctx->slots;
    std::vector<double> slots((size_t)C * w * S, 0.0);
    for (u32 c = 0; c < C; c++)
        for (u32 j = 0; j < w; j++) {
            double* z = &slots[((size_t)c * w + j) * S];
            for (u32 b = 0; b < B; b++)
                for (u32 i = 0; i < h; i++)
                    z[(size_t)b * Hp + pad + i] = x[(((size_t)b * C + c) * h + i) * w + j];
        }
    encrypt_slots_batch(ctx, ek, slots, C * w, level, seed_of(seed), first_ct_id, cols, ctx->stream);
    VR_HIP(hipStreamSynchronize(ctx->stream));
    API_END
}

vr_status vr_encrypt_matrix_columns(vr_context* ctx, const vr_eval_keys* ek, const double* M,
                                    uint32_t rows, uint32_t cols, uint32_t role, uint32_t m,
                                    uint32_t p, uint32_t level, const uint64_t* seed,
                                    uint64_t first_ct_id, vr_ciphertext** out)
{
    // outputs: role 0 cols, role 1 rows, role 2 T cols, role 3 rows, roles 4 / 5 nb
    u32 n_ct = role == 0 || role == 2 ? cols : rows;
    if (role == 2 && ctx && p >= 1 && p <= ctx->slots && m >= 1) {
        const u32 R = (u32)(ctx->slots / pow2ceil(p));
        n_ct = ((m + R - 1) / R) * cols;
    }
    u32 bPp = 0, bMb = 0, bc = 0, bnb = 0;
    if ((role == 4 || role == 5) && ctx && m >= 1 && p >= 1 && rows >= 1 && cols >= 1) {
        try {
            block_shape(ctx, m, role == 4 ? cols : rows, p, &bPp, &bMb, &bc, &bnb);
        } catch (const Error&) {
            bnb = 0;
        }
        n_ct = bnb;
    }
    if (out)
        for (u32 i = 0; i < n_ct; i++) out[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && M && out && seed, "null argument");
    REQUIRE(role <= 5, "role must be 0 (A columns), 1 (Bbar columns), 2 (A outer), 3 (B outer), "
                       "4 (A column blocks) or 5 (Bbar column blocks)");
    REQUIRE(rows >= 1 && cols >= 1 && m >= 1 && p >= 1, "empty matrix");
    REQUIRE(role == 0 || role == 2 || role == 4 ? rows == m : cols == p, "matrix shape does not match m / p");
    if (role >= 4) REQUIRE(bnb >= 1, "m + P' - 1 exceeds the slot count");
    REQUIRE(level <= ctx->L, "level above the modulus chain");
    const u32 Mp = pow2ceil(m), Pp = pow2ceil(p);
    REQUIRE(Pp <= ctx->slots && (role >= 2 || Mp <= ctx->slots), "matrix dimension exceeds the slot count");
    const size_t S = ctx->slots;
    const u32 R = (u32)(S / Pp);
    std::vector<double> slots((size_t)n_ct * S, 0.0);
    for (u32 c = 0; c < n_ct; c++) {
        double* z = &slots[(size_t)c * S];
        if (role == 2) {
            // A'_{t,k} (c = t cols + k): slot r P' + j -> A[t R + r][k], j < p
            const u32 t = c / cols, k = c - t * cols;
            for (u32 r = 0; r < R && (size_t)t * R + r < m; r++)
                for (u32 j = 0; j < p; j++) z[(size_t)r * Pp + j] = M[((size_t)t * R + r) * cols + k];
            continue;
        }
        if (role == 3) {
            // B'_k: slot r P' + j -> B[k][j], j < p, every row r
            for (u32 r = 0; r < R; r++)
                for (u32 j = 0; j < p; j++) z[(size_t)r * Pp + j] = M[(size_t)c * cols + j];
            continue;
        }
        if (role >= 4) {
            // column blocks: block j of ciphertext c holds column c bc + j of A
            // (role 4, first m slots) or row c bc + j of B (role 5, entry
            // r mod P' in slot r of the block)
            const u32 nn = role == 4 ? cols : rows;
            for (u32 j = 0; j < bc && (size_t)c * bc + j < nn; j++) {
                const u32 col = c * bc + j;
                double* blk = z + (size_t)j * bMb;
                if (role == 4)
                    for (u32 i = 0; i < m; i++) blk[i] = M[(size_t)i * cols + col];
                else
                    for (u32 r = 0; r < bMb; r++) blk[r] = r % bPp < p ? M[(size_t)col * cols + r % bPp] : 0.0;
            }
            continue;
        }
        const u32 k = c;
        for (size_t s = 0; s < S; s++) {
            if (role == 0) {
                u32 r = (u32)(s % Mp);
                z[s] = r < m ? M[(size_t)r * cols + k] : 0.0;
            } else {
                u32 r = (u32)(s % Pp);
                z[s] = r < p ? M[(size_t)k * cols + r] : 0.0;
            }
        }
    }
    encrypt_slots_batch(ctx, ek, slots, n_ct, level, seed_of(seed), first_ct_id, out, ctx->stream);
    VR_HIP(hipStreamSynchronize(ctx->stream));
    API_END
}

vr_status vr_rotate_batch(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* const* in,
                          size_t n, int32_t step, vr_ciphertext** outs, void* stream)
{
    if (outs)
        for (size_t i = 0; i < n; i++) outs[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && in && outs, "null argument");
    REQUIRE(n >= 1, "empty input");
    hipStream_t s = pick_stream(ctx, stream);
    Slab x = gather(ctx, in, (u32)n, s);
    REQUIRE(x.ncomp == 2, "rotation needs 2-component ciphertexts");
    std::vector<Slab> r;
    rotate_slab(ctx, ek, x, {step}, r, s);
    to_handles(ctx, r[0], outs);
    API_END
}

vr_status vr_matmul(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* const* A,
                    const vr_ciphertext* const* Bbar, uint32_t m, uint32_t n, uint32_t p,
                    vr_ciphertext** C, void* stream)
{
    const u32 Pp = m && p ? pow2ceil(std::min(m, p)) : 0;
    if (C)
        for (u32 i = 0; i < Pp; i++) C[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && A && Bbar && C, "null argument");
    REQUIRE(m >= 1 && n >= 1 && p >= 1, "empty matrix");
    hipStream_t s = pick_stream(ctx, stream);
    MatReq rq;
    rq.A = gather(ctx, A, n, s);
    rq.B = gather(ctx, Bbar, n, s);
    rq.m = m, rq.n = n, rq.p = p;
    std::vector<Slab> out = matmul_multi(ctx, ek, {rq}, s);
    to_handles(ctx, out[0], C);
    API_END
}

vr_status vr_matmul_block(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* const* A,
                          const vr_ciphertext* const* Bbar, uint32_t m, uint32_t n, uint32_t p,
                          vr_ciphertext** C, void* stream)
{
    const u32 Pp = p ? pow2ceil(p) : 0;
    if (C)
        for (u32 i = 0; i < Pp; i++) C[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && A && Bbar && C, "null argument");
    REQUIRE(m >= 1 && n >= 1 && p >= 1, "empty matrix");
    REQUIRE(m >= p, "the column-block form needs m >= p (multiply the transposes)");
    u32 bPp, Mb, c, nb;
    block_shape(ctx, m, n, p, &bPp, &Mb, &c, &nb);
    hipStream_t s = pick_stream(ctx, stream);
    MatReq rq;
    rq.A = gather(ctx, A, nb, s);
    rq.B = gather(ctx, Bbar, nb, s);
    rq.m = m, rq.n = nb, rq.p = p;
    Slab D = matmul_multi(ctx, ek, {rq}, s)[0];
    // fold the c blocks into block 0
    for (u32 t = 1; t < c; t <<= 1) {
        std::vector<Slab> r;
        rotate_slab(ctx, ek, D, {(int32_t)(Mb * t)}, r, s);
        launch_addsub(ctx, D.base, D.base, r[0].base, D.n * 2, D.level + 1, false, s);
    }
    to_handles(ctx, D, C);
    API_END
}

vr_status vr_matmul_plan(vr_context* ctx, uint32_t m, uint32_t n, uint32_t p, uint32_t level,
                         uint64_t max_client_cts, vr_matmul_cost* costs, uint32_t* chosen)
{
    if (chosen) *chosen = VR_MATMUL_NONE;
    API_BEGIN
    REQUIRE(ctx && costs && chosen, "null argument");
    REQUIRE(m >= 1 && n >= 1 && p >= 1, "empty matrix");
    REQUIRE(level >= 1 && level <= ctx->L, "level must leave one level for the rescale");
    // the column-split and column-block forms multiply the transposes when m < p
    const bool tr = m < p;
    const u32 mm = tr ? p : m, pp = tr ? m : p;
    KsShape k = ks_shape(ctx, level);
    const double nl = level + 1, ext = k.next;
    // device work in limb passes (one pass reads or writes N words): a
    // tensor reads four limbs and writes three per level; a key switch
    // transforms about 2 nl + beta (ext - alpha) + 2 (K + nl) limbs (two
    // passes each at the larger sizes), converts beta digits and the P part,
    // and reads beta digits plus the key for two outputs per extended limb
    const double tensor_pass = 7.0 * nl;
    const double ks_pass = 2.0 * (nl + k.beta * (ext - ctx->alpha) + 2.0 * (ctx->K + nl)) +
                           (k.beta * (ctx->alpha + ext) + 2.0 * (ctx->K + nl)) + (k.beta + 2.0) * ext +
                           2.0 * k.beta * ext;
    const double us_per_pass = (double)ctx->n * 8.0 / 5.0e12 * 1e6;   // 8N bytes at 5 TB/s effective
    for (int f = 0; f < 3; f++) costs[f] = vr_matmul_cost{};
    auto fill = [&](int f, double cts, double ks, double tens, int feasible) {
        costs[f].feasible = feasible;
        costs[f].transposed = f == VR_MATMUL_OUTER ? 0 : (tr ? 1 : 0);
        costs[f].client_cts = (uint64_t)cts;
        costs[f].key_switches = (uint64_t)ks;
        costs[f].tensors = (uint64_t)tens;
        costs[f].est_us = (ks * ks_pass + tens * tensor_pass) * us_per_pass;
    };
    {
        const double P1 = pow2ceil(pp);
        const bool ok = pow2ceil(mm) <= ctx->slots;
        fill(VR_MATMUL_COLUMN_SPLIT, 2.0 * n, n * (P1 - 1) + P1, n * P1, ok ? 1 : 0);
    }
    {
        u32 bP, Mb, c, nb;
        bool ok = true;
        try {
            block_shape(ctx, mm, n, pp, &bP, &Mb, &c, &nb);
        } catch (const Error&) {
            ok = false, bP = 1, Mb = 1, c = 1, nb = n;
        }
        double lc = 0;
        for (u32 t = 1; t < c; t <<= 1) lc += 1;
        fill(VR_MATMUL_COLUMN_BLOCK, 2.0 * nb, nb * (bP - 1.0) + bP * lc + bP, (double)nb * bP, ok ? 1 : 0);
    }
    {
        const u32 P1 = pow2ceil(p);
        const bool ok = P1 <= ctx->slots;
        const double R = ok ? (double)(ctx->slots / P1) : 1.0, T = std::ceil(m / R);
        fill(VR_MATMUL_OUTER, T * n + n, T, T * n, ok ? 1 : 0);
    }
    int best = -1;
    for (int f = 0; f < 3; f++) {
        if (!costs[f].feasible || (max_client_cts && costs[f].client_cts > max_client_cts)) continue;
        if (best < 0 || costs[f].est_us < costs[best].est_us) best = f;
    }
    REQUIRE(best >= 0, "no form fits the client ciphertext limit");
    *chosen = (uint32_t)best;
    API_END
}

vr_status vr_matmul_outer(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* const* A,
                          const vr_ciphertext* const* B, uint32_t m, uint32_t n, uint32_t p,
                          vr_ciphertext** C, void* stream)
{
    u32 T = 0;
    if (ctx && m >= 1 && p >= 1 && pow2ceil(p) <= ctx->slots) {
        const u32 R = (u32)(ctx->slots / pow2ceil(p));
        T = (m + R - 1) / R;
    }
    if (C)
        for (u32 i = 0; i < T; i++) C[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && A && B && C, "null argument");
    REQUIRE(m >= 1 && n >= 1 && p >= 1, "empty matrix");
    u32 Pp, R, Tt;
    outer_tiles(ctx, m, p, &Pp, &R, &Tt);
    hipStream_t s = pick_stream(ctx, stream);
    MatReq rq;
    rq.A = gather(ctx, A, Tt * n, s);
    rq.B = gather(ctx, B, n, s);
    rq.m = m, rq.n = n, rq.p = p;
    std::vector<Slab> out = matmul_outer_multi(ctx, ek, {rq}, s);
    to_handles(ctx, out[0], C);
    API_END
}

vr_status vr_conv2d(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* const* in,
                    uint32_t C_in, uint32_t h, uint32_t w, uint32_t pad, const double* K,
                    const double* bias, uint32_t C_out, uint32_t k, uint32_t stride,
                    vr_ciphertext** out, void* stream)
{
    return vr_conv2d_sets(ctx, ek, in, 1, C_in, h, w, pad, K, bias, C_out, k, stride, out, stream);
}

vr_status vr_conv2d_sets(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* const* in,
                         uint32_t n_sets, uint32_t C_in, uint32_t h, uint32_t w, uint32_t pad,
                         const double* K, const double* bias, uint32_t C_out, uint32_t k,
                         uint32_t stride, vr_ciphertext** out, void* stream)
{
    const u32 wo = (k >= 1 && stride >= 1 && w + 2 * pad >= k) ? (w + 2 * pad - k) / stride + 1 : 0;
    if (out)
        for (size_t i = 0; i < (size_t)n_sets * C_out * wo; i++) out[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && in && K && bias && out, "null argument");
    REQUIRE(n_sets >= 1, "no image set");
    REQUIRE(C_in >= 1 && C_out >= 1 && k >= 1 && stride >= 1, "bad conv shape");
    REQUIRE(w + 2 * pad >= k && h + 2 * pad >= k, "kernel larger than the padded image");
    REQUIRE(pad < k, "padding must be smaller than the kernel");
    hipStream_t s = pick_stream(ctx, stream);
    Slab x = gather(ctx, in, n_sets * C_in * w, s);
    Slab y = conv_slab(ctx, ek, x, n_sets, C_in, w, pad, K, bias, C_out, k, stride, s);
    to_handles(ctx, y, out);
    API_END
}

vr_status vr_square(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* const* in,
                    size_t n, vr_ciphertext** out, void* stream)
{
    if (out)
        for (size_t i = 0; i < n; i++) out[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && in && out, "null argument");
    REQUIRE(n >= 1, "empty input");
    hipStream_t s = pick_stream(ctx, stream);
    Slab x = gather(ctx, in, (u32)n, s);
    Slab y = square_slab(ctx, ek, x, s);
    to_handles(ctx, y, out);
    API_END
}

vr_status vr_encode_fc_weights(vr_context* ctx, const double* W, uint32_t n_out, uint32_t C,
                               uint32_t h_out, uint32_t w_out, uint32_t stride, uint32_t block,
                               uint32_t level, vr_plaintext** W_pt)
{
    const size_t total = (size_t)n_out * C * w_out;
    if (W_pt)
        for (size_t i = 0; i < total; i++) W_pt[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && W && W_pt, "null argument");
    REQUIRE(n_out >= 1 && C >= 1 && h_out >= 1 && w_out >= 1 && stride >= 1, "empty FC layer");
    REQUIRE(block >= 1 && (block & (block - 1)) == 0 && block <= ctx->slots, "block must be a power of two <= S");
    REQUIRE((size_t)stride * (h_out - 1) < block, "rows do not fit the block");
    REQUIRE(level <= ctx->L, "level above the modulus chain");
    hipStream_t s = ctx->stream;
    const size_t S = ctx->slots, N = ctx->n;
    const u32 nl = level + 1;
    const u32 nb = (u32)(S / block);
    std::vector<double> slots(total * S, 0.0);
    for (u32 o = 0; o < n_out; o++)
        for (u32 c = 0; c < C; c++)
            for (u32 jo = 0; jo < w_out; jo++) {
                double* z = &slots[(((size_t)o * C + c) * w_out + jo) * S];
                for (u32 b = 0; b < nb; b++)
                    for (u32 i = 0; i < h_out; i++)
                        z[(size_t)b * block + (size_t)stride * i] = W[(((size_t)o * C + c) * h_out + i) * w_out + jo];
            }
    const double sc = (double)ctx->mod[level];
    BufPtr xd = dev_alloc(ctx, slots.size() * sizeof(double), s);
    VR_HIP(hipMemcpyAsync(xd->ptr, slots.data(), slots.size() * sizeof(double), hipMemcpyHostToDevice, s));
    BufPtr mb = dev_alloc(ctx, total * nl * N * sizeof(u64), s);
    // the slot vectors repeat with period `block`: encoded in Z[X^r],
    // r = N / (2 block), and in the evaluation domain (bit-reversed order)
    // every limb then repeats in runs of r consecutive words
    u32 rep = 0;
    while ((2ull * block) << (rep + 1) <= N) rep++;
    encode_to_limbs(ctx, (const double*)xd->ptr, (u32)S, (u32)total, S, sc, as_u64(mb), nl,
                    (u64)nl * N, s, rep);
    ntt_forward(ctx, poly_limbs(as_u64(mb), as_u64(mb), (u32)total, nl, (u64)nl * N, (int)level), s);
    BufPtr cb;
    if (rep > 0) {
        // one compact copy of all of them, checked word for word
        const size_t cn = N >> rep;
        cb = dev_alloc(ctx, total * nl * cn * sizeof(u64), s);
        BufPtr flag = dev_alloc(ctx, sizeof(int), s);
        VR_HIP(hipMemsetAsync(flag->ptr, 0, sizeof(int), s));
        dim3 grid((u32)((cn + kThreads - 1) / kThreads), (u32)(total * nl));
        hipLaunchKernelGGL(k_compact_runs, grid, dim3(kThreads), 0, s, as_u64(mb), as_u64(cb), ctx->log_n, rep,
                           (int*)flag->ptr);
        VR_CHECK_LAUNCH();
        int bad = 0;
        VR_HIP(hipMemcpyAsync(&bad, flag->ptr, sizeof(int), hipMemcpyDeviceToHost, s));
        VR_HIP(hipStreamSynchronize(s));
        if (bad) cb.reset();
    }
    for (size_t i = 0; i < total; i++) {
        auto* pt = new vr_plaintext;
        pt->ctx = ctx;
        pt->buf = mb;
        pt->data = as_u64(mb) + i * nl * N;
        pt->level = level;
        pt->scale = sc;
        if (cb) {
            pt->cbuf = cb;
            pt->cdata = as_u64(cb) + i * nl * (N >> rep);
            pt->clog = rep;
        }
        W_pt[i] = pt;
    }
    VR_HIP(hipStreamSynchronize(s));
    API_END
}

vr_status vr_conv2d_encw(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* const* in, uint32_t C_in,
                         uint32_t h, uint32_t w, uint32_t pad, const vr_ciphertext* const* K_ct,
                         const vr_ciphertext* const* bias_ct, uint32_t C_out, uint32_t k, uint32_t stride,
                         vr_ciphertext** out, void* stream)
{
    const u32 wo = (k >= 1 && stride >= 1 && w + 2 * pad >= k) ? (w + 2 * pad - k) / stride + 1 : 0;
    if (out)
        for (u32 i = 0; i < C_out * wo; i++) out[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && in && K_ct && bias_ct && out, "null argument");
    REQUIRE(C_in >= 1 && C_out >= 1 && k >= 1 && stride >= 1 && pad < k && wo >= 1 && h + 2 * pad >= k,
            "bad conv shape");
    hipStream_t s = pick_stream(ctx, stream);
    Slab x = gather(ctx, in, C_in * w, s);
    Slab Kw = gather(ctx, K_ct, C_out * C_in * k * k, s);
    Slab B = gather(ctx, bias_ct, C_out, s);
    Slab y = conv_encw_slab(ctx, ek, x, C_in, w, pad, Kw, B, C_out, k, stride, s);
    to_handles(ctx, y, out);
    API_END
}

vr_status vr_fc_encw(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* const* Y, uint32_t n_in,
                     const vr_ciphertext* const* W_ct, const vr_ciphertext* const* bias_ct, uint32_t n_out,
                     uint32_t block, vr_ciphertext** out, void* stream)
{
    if (out)
        for (u32 i = 0; i < n_out; i++) out[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && Y && W_ct && bias_ct && out && n_in >= 1 && n_out >= 1, "null argument");
    REQUIRE(block >= 1 && (block & (block - 1)) == 0 && block <= ctx->slots, "block must be a power of two <= S");
    hipStream_t s = pick_stream(ctx, stream);
    Slab y = gather(ctx, Y, n_in, s);
    Slab Wc = gather(ctx, W_ct, n_out * n_in, s);
    Slab B = gather(ctx, bias_ct, n_out, s);
    Slab z = fc_encw_slab(ctx, ek, y, Wc, B, n_out, block, s);
    to_handles(ctx, z, out);
    API_END
}

vr_status vr_poly_eval(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* const* in, size_t n,
                       const double* coeffs, uint32_t degree, vr_ciphertext** out, void* stream)
{
    if (out)
        for (size_t i = 0; i < n; i++) out[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && in && coeffs && out && n >= 1, "null argument");
    REQUIRE(degree >= 1, "degree must be at least 1");
    hipStream_t s = pick_stream(ctx, stream);
    Slab x = gather(ctx, in, (u32)n, s);
    Slab y = poly_slab(ctx, ek, x, coeffs, degree, s);
    to_handles(ctx, y, out);
    API_END
}

vr_status vr_dense(vr_context* ctx, const vr_ciphertext* const* in, uint32_t n_in, const double* W,
                   const double* bias, uint32_t n_out, vr_ciphertext** out, void* stream)
{
    if (out)
        for (u32 i = 0; i < n_out; i++) out[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && in && W && bias && out && n_in >= 1 && n_out >= 1, "null argument");
    hipStream_t s = pick_stream(ctx, stream);
    Slab z = gather(ctx, in, n_in, s);
    Slab y = dense_slab(ctx, z, W, bias, n_out, s);
    to_handles(ctx, y, out);
    API_END
}

vr_status vr_fc(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* const* Y, uint32_t C,
                uint32_t w_out, const vr_plaintext* const* W_pt, const double* bias, uint32_t n_out,
                uint32_t block, vr_ciphertext** out, void* stream)
{
    if (out)
        for (u32 i = 0; i < n_out; i++) out[i] = nullptr;
    API_BEGIN
    REQUIRE(ctx && ek && Y && W_pt && bias && out, "null argument");
    REQUIRE(C >= 1 && w_out >= 1 && n_out >= 1, "empty FC layer");
    REQUIRE(block >= 1 && (block & (block - 1)) == 0 && block <= ctx->slots, "block must be a power of two <= S");
    hipStream_t s = pick_stream(ctx, stream);
    const u32 n_in = C * w_out;
    Slab y = gather(ctx, Y, n_in, s);
    REQUIRE(y.ncomp == 2, "FC inputs must be 2-component");
    BufPtr hold;
    u64 p_stride = 0;
    double p_scale = 0;
    u32 p_level = 0;
    u32 p_rep = 0;
    const u64* P = fc_weights(ctx, W_pt, (size_t)n_out * n_in, y.level + 1, &p_stride, &p_scale, &p_level,
                              hold, s, &p_rep);
    Slab z = fc_slab(ctx, ek, y, P, p_stride, p_scale, p_level, n_out, bias, block, s, p_rep);
    to_handles(ctx, z, out);
    API_END
}

}  // extern "C"
