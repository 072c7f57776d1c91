// Launchers for the element-wise, rescale, automorphism, base-conversion,
// key-switching, sampling and FFT kernels.  All polynomials are in the
// evaluation domain unless a name says "coef".  `nl` is the number of limbs
// per polynomial (level + 1 for Q-chain polynomials); limb l of every poly
// uses modulus index l.
#pragma once

#include "vr_core.h"

namespace vr {

// per-limb scalar constants with Shoup companions (kernel argument)
struct LimbConsts {
    u64 c[kMaxMod];
    u64 cs[kMaxMod];
};
VR_KERNEL_ARG(LimbConsts);

// out = a (+|-) b over n_polys x nl limbs (dense [n_polys][nl][N]).
void launch_addsub(vr_context* ctx, u64* out, const u64* a, const u64* b, u32 n_polys, u32 nl,
                   bool sub, hipStream_t s);
// out[p][l] = a[p][l] * c[l]  (Shoup)
void launch_mul_scalar(vr_context* ctx, u64* out, const u64* a, u32 n_polys, u32 nl,
                       const LimbConsts& c, hipStream_t s);
// out[l] = a[l] + c[l] on every slot of one polynomial
void launch_add_scalar(vr_context* ctx, u64* out, const u64* a, u32 nl, const LimbConsts& c,
                       hipStream_t s);
// out[p][l] = a[p][l] * pt[l]
void launch_mul_plain(vr_context* ctx, u64* out, const u64* a, const u64* pt, u32 n_polys, u32 nl,
                      hipStream_t s);
// out (3 polys) = (a0 b0, a0 b1 + a1 b0, a1 b1)
void launch_tensor(vr_context* ctx, u64* out, const u64* a, const u64* b, u32 nl, hipStream_t s);
// out[l] = a[perm_g(l slots)] : Galois automorphism X -> X^g in the evaluation domain
void launch_automorphism(vr_context* ctx, u64* out, const u64* a, u32 n_polys, u32 nl,
                         u64 poly_stride, u32 g, hipStream_t s);
// coef[k] (centred modulo q_level) -> r[k][i] = [coef]_{q_i}, i < level (dense)
void launch_rescale_spread(vr_context* ctx, u64* r, const u64* coef, u32 n_polys, u32 level,
                           hipStream_t s);
// out[k][i] = (c[k][i] - r[k][i]) * q_level^-1, i < level
void launch_rescale_finish(vr_context* ctx, u64* out, const u64* c, const u64* r, u32 n_polys,
                           u32 level, hipStream_t s);
// rows x width words: dst + r * dst_stride <- src + r * src_stride (device to device)
void launch_copy_rows(u64* dst, u64 dst_stride, const u64* src, u64 src_stride, u64 width, u32 rows,
                      hipStream_t s);
// signed integer coefficients x[N] -> limbs [n_mods][N] at modulus indices mods[]
void launch_int_to_limbs(vr_context* ctx, u64* out, const i64* x, const u32* mods_host, u32 n_mods,
                         hipStream_t s);

// ---------------------------------------------------------- key switching

// Scratch needed by one key switch at `level` (bytes).
struct KsShape {
    u32 level, nq, next, beta;
};
KsShape ks_shape(vr_context* ctx, u32 level);

// ModUp of d (evaluation domain, nq limbs): X = [beta][next][N] extended digits
// in the evaluation domain, except each digit's own limbs (rows j next + i,
// i in digit j), which are d itself and are not written: the inner product
// reads them from d.  Uses `coef` ([nq][N]) as scratch.
void keyswitch_modup(vr_context* ctx, const u64* d, u32 level, u64* X, u64* coef, hipStream_t s);
// Batched ModUp: d_c = d + c*d_stride (c < n_ct), X_c = X + c*beta*next*N,
// coef: [n_ct][nq][N] scratch.
// keep_q > 0 (digits of more than one limb): only the extended limbs
// q_0..q_{keep_q-1}, q_level and the special primes of X are made (the ones a
// keep_q inner product reads); the rest of X is left as it was.
void keyswitch_modup_batch(vr_context* ctx, const u64* d, u64 d_stride, u32 n_ct, u32 level,
                           u64* X, u64* coef, hipStream_t s, u32 keep_q = 0);
// U = [2][next][N]: sum_j sigma_g(X_j) * (b_j, a_j) (g = 1: no automorphism);
// d is the ModUp input (the digits' own limbs).
void keyswitch_inner(vr_context* ctx, const u64* X, const u64* d, const u64* key, u32 level, u32 g,
                     u64* U, hipStream_t s);
// Batched inner product: n_ct digit sets X + c*x_stride (ModUp inputs
// d + c*d_stride) share one key read.  With fold_c0 (ciphertext c's c0 at
// fold_c0 + c*fold_stride, level limbs) the Q limbs of U_0 also take
// P sigma_g(c0): U is then P times the rotation before its ModDown.  With
// keep_q > 0 only the limbs q_0..q_{keep_q-1}, q_level and the special primes
// are computed, and U holds them compactly in that order ([2][keep_q+1+K][N]
// per ciphertext).
void keyswitch_inner_batch(vr_context* ctx, const u64* X, u64 x_stride, const u64* d, u64 d_stride,
                           u32 n_ct, const u64* key, u32 level, u32 g, u64* U, u64 u_stride,
                           hipStream_t s, const u64* fold_c0 = nullptr, u64 fold_stride = 0,
                           u32 keep_q = 0);
// The same for two rotation steps at once (keys key0/key1, Galois elements
// g0/g1, outputs U0/U1 with one stride): each digit word is read once.
void keyswitch_inner_batch2(vr_context* ctx, const u64* X, u64 x_stride, const u64* d, u64 d_stride,
                            u32 n_ct, const u64* key0, const u64* key1, u32 level, u32 g0, u32 g1, u64* U0,
                            u64* U1, u64 u_stride, hipStream_t s, const u64* fold_c0 = nullptr,
                            u64 fold_stride = 0, u32 keep_q = 0);
// ModDown of U ([2][next][N]) to out0/out1 (nq limbs each, may be strided),
// adding add0 (optionally through sigma_g) and add1 when non-null.
void keyswitch_moddown(vr_context* ctx, u64* U, u32 level, u64* out0, u64* out1, const u64* add0,
                       u32 add0_g, const u64* add1, u64* scratch, hipStream_t s);
// Batched ModDown: n_ct independent U blocks (u_stride apart), outputs out0 +
// c*out_stride etc.
void keyswitch_moddown_batch(vr_context* ctx, u64* U, u64 u_stride, u32 n_ct, u32 level,
                             u64* out0, u64* out1, u64 out_stride, const u64* add0, u32 add0_g,
                             const u64* add1, u64 add_stride, u64* scratch, hipStream_t s);
// Relinearisation fused with the rescale: ModDown of U by P q_l (l = level)
// with c0/c1 (the ciphertext's first two components, level l, c_stride apart
// per ciphertext) folded in (both null: U is taken as it is); out0/out1 get
// l limbs (level l - 1).  Scratch as keyswitch_moddown_scratch(level, n_ct).
// keep_q > 0: U is the compact layout of keyswitch_inner_batch's keep_q and
// only output limbs 0..keep_q-1 are made (level keep_q - 1).
void keyswitch_moddown_rescale_batch(vr_context* ctx, u64* U, u64 u_stride, u32 n_ct, u32 level,
                                     u64* out0, u64* out1, u64 out_stride, const u64* c0,
                                     const u64* c1, u64 c_stride, u64* scratch, hipStream_t s,
                                     u32 keep_q = 0);
// scratch sizes in u64 words
size_t keyswitch_modup_scratch(vr_context* ctx, u32 level);     // X + coef
size_t keyswitch_moddown_scratch(vr_context* ctx, u32 level, u32 n_ct);

// ---------------------------------------------------------- sampling

// The 256-bit ChaCha20 key of every sample: w[0] holds key bytes 0..7
// (little-endian), w[3] bytes 24..31.
struct Seed256 {
    u64 w[4];
};
VR_KERNEL_ARG(Seed256);
inline Seed256 seed_of(const uint64_t* w)
{
    Seed256 s;
    for (int i = 0; i < 4; i++) s.w[i] = w[i];
    return s;
}

enum Purpose : u32 {
    kPurSk = 1, kPurPkA = 2, kPurPkE = 3, kPurSwkA = 4, kPurSwkE = 5,
    kPurEncV = 6, kPurEncE0 = 7, kPurEncE1 = 8
};
void launch_sample_ternary(vr_context* ctx, i64* out, const Seed256& seed, u32 purpose, u64 obj, hipStream_t s);
void launch_sample_gauss(vr_context* ctx, i64* out, const Seed256& seed, u32 purpose, u64 obj, hipStream_t s);
// limbs [n][N] (coefficient domain): limb i uses stream limb index limb_index[i]
// and modulus index mods[i]
void launch_sample_uniform(vr_context* ctx, u64* out, const Seed256& seed, u32 purpose, u64 obj,
                           const u32* limb_index_host, const u32* mods_host, u32 n, hipStream_t s);

// keygen / encryption combiners (evaluation domain)
// b = -a*s + e (+ [P]_q * sp on limbs in [dlo, dhi)); limb l is modulus index l
void launch_key_combine(vr_context* ctx, u64* b, const u64* a, const u64* e, const u64* s_all,
                        const u64* sp_all, u32 n, u32 dlo, u32 dhi, hipStream_t st);
// c0 = v*pk_b + e0 + m, c1 = v*pk_a + e1 over nl limbs
void launch_encrypt_combine(vr_context* ctx, u64* ct, const u64* v, const u64* e0, const u64* e1,
                            const u64* pk, const u64* m, u32 nl, hipStream_t s);
// m = c0 + c1 s (+ c2 s^2)
void launch_decrypt_combine(vr_context* ctx, u64* m, const u64* ct, u32 ncomp, const u64* s_all,
                            u32 nl, hipStream_t s);

// ---------------------------------------------------------- encode / decode

// slots x[n] (n <= S) at `scale` -> integer coefficients reduced into nl limbs
// (coefficient domain); sub_log > 0: the slots repeat with period S / 2^sub_log
// and the coefficients off the subring Z[X^(2^sub_log)] (FFT noise) are zero
void encode_to_limbs(vr_context* ctx, const double* x_dev, u32 n, u32 n_vec, u64 vec_stride_x,
                     double scale, u64* limbs, u32 nl, u64 limbs_stride, hipStream_t s, u32 sub_log = 0);
// limb q_0 coefficients (coefficient domain) -> slots out[n] / scale
void decode_from_limb0(vr_context* ctx, const u64* coef0, double scale, double* out_dev, u32 n,
                       hipStream_t s);

}  // namespace vr
