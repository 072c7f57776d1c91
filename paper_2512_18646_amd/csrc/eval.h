// Internal evaluator: the HE operations on handles, shared by the C ABI and
// the layer schedules.  Every function enqueues on `s` and returns a new
// handle (caller owns it); errors are thrown as vr::Error.
#pragma once

#include "vr_ops.h"

namespace vr {

void build_context(vr_context* ctx, const vr_params* p, int device);

// The no-allocation rotation's fixed device array (per GPU): its size, the
// words a rotation at `level` takes from it, and its registration (device
// address taken once per device, that device current).
constexpr size_t kNoAllocScratchBytes = size_t(144) << 20;
size_t noalloc_rotate_words(vr_context* ctx, u32 level);
void noalloc_register_device(int device);
void destroy_context_tables(vr_context* ctx);

inline hipStream_t pick_stream(vr_context* ctx, void* s) { return s ? (hipStream_t)s : ctx->stream; }

vr_ciphertext* new_ct(vr_context* ctx, u32 ncomp, u32 level, double scale, hipStream_t s);
vr_plaintext* new_pt(vr_context* ctx, u32 level, double scale, hipStream_t s);
// view into an existing buffer (shares ownership)
vr_ciphertext* view_ct(vr_context* ctx, const BufPtr& buf, u64* data, u32 ncomp, u32 level,
                       double scale);

u32 galois_element(vr_context* ctx, int32_t step);
// [round-half-away(x)]_q for any finite double x, exact
u64 double_to_mod(double x, u64 q);

void check_same(const vr_ciphertext* a, const vr_ciphertext* b);
const vr_switch_key& rot_key(const vr_eval_keys* ek, u32 g);

vr_ciphertext* ev_add(vr_context* ctx, const vr_ciphertext* a, const vr_ciphertext* b, bool sub,
                      hipStream_t s);
vr_ciphertext* ev_mul_const(vr_context* ctx, const vr_ciphertext* a, double c, double c_scale,
                            hipStream_t s);
vr_ciphertext* ev_add_const(vr_context* ctx, const vr_ciphertext* a, double c, hipStream_t s);
vr_ciphertext* ev_mul_plain(vr_context* ctx, const vr_ciphertext* a, const vr_plaintext* pt,
                            hipStream_t s);
vr_ciphertext* ev_tensor(vr_context* ctx, const vr_ciphertext* a, const vr_ciphertext* b,
                         hipStream_t s);
// Relinearisation and rescale in one ModDown by P q_l (level l - 1).
vr_ciphertext* ev_relin_rescale(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* a,
                                hipStream_t s);
vr_ciphertext* ev_relin(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* a,
                        hipStream_t s);
vr_ciphertext* ev_rescale(vr_context* ctx, const vr_ciphertext* a, hipStream_t s);
vr_ciphertext* ev_mod_drop(vr_context* ctx, const vr_ciphertext* a, u32 level, hipStream_t s);
void ev_rotate_many(vr_context* ctx, const vr_eval_keys* ek, const vr_ciphertext* a,
                    const int32_t* steps, size_t k, vr_ciphertext** outs, hipStream_t s);

vr_plaintext* ev_encode(vr_context* ctx, const double* x_host, size_t n, u32 level, double scale,
                        hipStream_t s);
vr_ciphertext* ev_encrypt(vr_context* ctx, const vr_eval_keys* ek, const vr_plaintext* pt,
                          const Seed256& seed, u64 ct_id, hipStream_t s);

// rescale of n_ct ciphertexts laid out densely (stride = ncomp*(level+1)*N) into out
void rescale_dense(vr_context* ctx, const u64* in, u64* out, u32 n_polys, u32 level, hipStream_t s);

}  // namespace vr
