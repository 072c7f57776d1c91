// Slabs: a layer's ciphertexts in one allocation, so one kernel launch covers
// all of them.  Shared by the layer calls and the serving loop.
#pragma once

#include "eval.h"

namespace vr {

struct Slab {
    BufPtr buf;
    u64* base = nullptr;
    u32 n = 0, ncomp = 2, level = 0;
    u32 ext = 0;      // 1: P times 2-component ciphertexts over q_0..q_level, p_0..p_{K-1}
    u32 keep = 0;     // ext with keep > 0: only q_0..q_{keep-1}, q_level, p_0..p_{K-1}
    u64 stride = 0;   // words between ciphertexts
    double scale = 1.0;
    u64* ct(u32 i) const { return base + (size_t)i * stride; }
};

Slab new_slab(vr_context* ctx, u32 n, u32 ncomp, u32 level, double scale, hipStream_t s);
// n ciphertexts in the extended basis (level + 1 + K limbs per component, or
// keep + 1 + K with keep > 0: q_0..q_{keep-1}, q_level, the special primes)
Slab new_ext_slab(vr_context* ctx, u32 n, u32 level, double scale, hipStream_t s, u32 keep = 0);
// the ciphertexts in place when they already form a slab, else a copy
Slab gather(vr_context* ctx, const vr_ciphertext* const* cts, u32 n, hipStream_t s);
// new handles viewing the slab's ciphertexts (they share its allocation)
void to_handles(vr_context* ctx, const Slab& sl, vr_ciphertext** out);

// Ciphertexts [begin, end) of a slab key-switch with the keys of ek (one
// session's share of a serving wave).
struct KeyRange {
    u32 begin, end;
    const vr_eval_keys* ek;
};

// conv layer over n_sets image sets (set s: ciphertexts s*C_in*w ...)
Slab conv_slab(vr_context* ctx, const vr_eval_keys* ek, const Slab& x, u32 n_sets, u32 C_in, u32 w,
               u32 pad, const double* K, const double* bias, u32 C_out, u32 k, u32 stride,
               hipStream_t s);
// x^2 of every ciphertext: Rescale(Relin(Tensor(y, y)))
Slab layer_square(vr_context* ctx, const vr_eval_keys* ek, const Slab& in, hipStream_t s);
// FC layer: Z_o = RotSum_block(Rescale(sum_i y_i * P[o][i])) + bias_o with the
// weight plaintexts P[o][i] at P + (o * y.n + i) * p_stride, evaluated at
// min(y.level, p_level) (inputs above the weights' level are read on its limbs)
// p_rep > 0: the weights are compact copies (runs of 2^p_rep equal words kept
// once, N >> p_rep words per limb)
Slab fc_slab(vr_context* ctx, const vr_eval_keys* ek, const Slab& y, const u64* P, u64 p_stride,
             double p_scale, u32 p_level, u32 n_out, const double* bias, u32 block, hipStream_t s,
             u32 p_rep = 0);
// A network (conv, optional x^2, optional FC) with its constants resolved.
struct CnnDesc {
    u32 C_in, h, w, pad, C_out, k, stride, square;
    std::vector<double> K, bias, fc_bias;
    std::vector<BufPtr> fc_hold;     // keeps the weight plaintexts alive
    const u64* fc_P = nullptr;
    u64 fc_stride = 0;
    double fc_scale = 0;
    u32 fc_level = 0;                // level the FC runs at (its weights' level or below)
    u32 fc_rep = 0;                  // weights compact (runs of 2^fc_rep words kept once)
    u32 fc_out = 0, fc_block = 0;
    u32 w_out() const { return (w + 2 * pad - k) / stride + 1; }
    u32 n_in() const { return C_in * w; }
    u32 n_out() const { return fc_out ? fc_out : C_out * w_out(); }
    u32 levels() const { return 1 + square + (fc_out ? 1 : 0); }
};
CnnDesc make_desc(vr_context* ctx, const vr_cnn_desc* d, u32 level_in, hipStream_t s);
// One segment of a serving wave: n_sets image sets of network d under the
// keys of one session.
struct NetSeg {
    const CnnDesc* d;
    const vr_eval_keys* ek;
    u32 n_sets;
};
// Every segment's network over the slab x, which holds the segments' input
// columns back to back.  Networks and sessions may differ; the segments must
// share the conv kernel size, the x^2 flag, FC presence and the FC level,
// and FC segments come in decreasing block order.  The stages whose keys do
// not matter (ModUp, ModDown, NTTs, rescale, tensor) run once over all
// segments, the inner products per session, the linear combinations and
// weight products per network.  Outputs segment after segment, set after set.
Slab run_cnn_multi(vr_context* ctx, const std::vector<NetSeg>& segs, const Slab& x, hipStream_t s);
// the network on n_sets image sets (slab x, set after set); outputs set after set
Slab run_cnn(vr_context* ctx, const vr_eval_keys* ek, const CnnDesc& d, const Slab& x, u32 n_sets,
             hipStream_t s);

// One column-split product C = A B (A_k, Bbar_k column slabs of n each).
struct MatReq {
    Slab A, B;
    u32 m = 0, n = 0, p = 0;
};
// Products of several requests at one level and scale, sharing the hoisted
// ModUp and each rotation step's key; result r holds P'_r ciphertexts.
std::vector<Slab> matmul_multi(vr_context* ctx, const vr_eval_keys* ek, const std::vector<MatReq>& reqs,
                               hipStream_t s);
// Outer-product products (A: T n ciphertexts, tile-major; B: n) at one level
// and scale: every request's tiles relinearised and rescaled together;
// result r holds T_r ciphertexts.
std::vector<Slab> matmul_outer_multi(vr_context* ctx, const vr_eval_keys* ek, const std::vector<MatReq>& reqs,
                                     hipStream_t s);
// (P', R, T) of the outer-product form: column padding, rows per ciphertext, tiles
void outer_tiles(vr_context* ctx, u32 m, u32 p, u32* Pp, u32* R, u32* T);
// (P', Mb, c, nb) of the column-block form: block size, columns per
// ciphertext, ciphertexts per operand
void block_shape(vr_context* ctx, u32 m, u32 n, u32 p, u32* Pp, u32* Mb, u32* c, u32* nb);
// Weight plaintexts as one array of count plaintexts; *p_level = the level
// the layer runs at, min(nl - 1, the plaintexts' level).
// *p_rep > 0: the returned weights are the plaintexts' compact copies
const u64* fc_weights(vr_context* ctx, const vr_plaintext* const* W_pt, size_t count, u32 nl,
                      u64* p_stride, double* p_scale, u32* p_level, BufPtr& holder, hipStream_t s,
                      u32* p_rep);

}  // namespace vr
