// Internal header of the HIP library: device modular arithmetic, context and
// object layouts, and the launchers every translation unit shares.
//
// Data layout in HBM (all uint64, limb-major, coefficient index fastest so
// every wavefront reads 64 consecutive words of one limb):
//   ciphertext   [ncomp][level+1][N]   evaluation (NTT) domain
//   plaintext    [level+1][N]          evaluation domain
//   switch key   [dnum][2][L+1+K][N]   (b_j then a_j; limbs q_0..q_L, p_0..p_{K-1})
//   public key   [2][L+1][N]
// Modulus index m: 0..L are the Q chain, L+1..L+K the special primes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <array>
#include <atomic>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/vr.h"
#include "alloc.h"

namespace vr {

typedef uint64_t u64;
typedef int64_t i64;
typedef uint32_t u32;
typedef unsigned __int128 u128;

// Moduli per context (Q chain + special primes).  Per-limb constant tables
// passed by value to kernels are sized by it (2 x 40 x 8 = 640 bytes).
constexpr int kMaxMod = 40;

// Budget for a struct passed by value to a kernel.  Keys generated with two
// 1 KiB tables among the arguments (2 KiB in all) came out wrong on limbs past
// the first; the cause was not found, so every by-value argument struct is
// held to this size (static_assert beside each), leaving room under 1 KiB for
// the kernel's pointers and scalars, and larger per-limb tables live in
// device memory.
constexpr unsigned kMaxArgStruct = 896;
#define VR_KERNEL_ARG(T) \
    static_assert(sizeof(T) <= kMaxArgStruct, #T " is passed by value to kernels: keep it under the budget")

// --------------------------------------------------------------- errors

struct Error : std::runtime_error {
    vr_status code;
    Error(vr_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define VR_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw ::vr::Error(VR_EDEVICE, std::string(#call " failed: ") + hipGetErrorString(e_)); \
    } while (0)

#define VR_CHECK_LAUNCH() VR_HIP(hipGetLastError())

// ------------------------------------------------- per-modulus constants

// Everything a kernel needs to reduce modulo one prime q < 2^61.
struct ModQ {
    u64 q;
    u64 mu;      // floor(2^(2k) / q), Barrett constant for products < q^2
    u64 r64;     // 2^64 mod q
    u64 r64_s;   // floor(r64 * 2^64 / q)  (Shoup companion)
    u64 one_s;   // floor(2^64 / q)
    u64 ninv;    // N^-1 mod q
    u64 ninv_s;
    u64 inw1;    // N^-1 times the inverse transform's last-stage twiddle, mod q
    u64 inw1_s;
    u64 pmod;    // P = prod of the special primes, mod q
    u64 pmod_s;
    u64 pinv;    // P^-1 mod q (Q-chain moduli only)
    u64 pinv_s;
    u32 k;       // bit length of q
    u32 pad_;
};

__host__ __device__ inline u64 shoup_companion(u64 w, u64 q)
{
    return (u64)(((u128)w << 64) / q);
}

#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)
__device__ __forceinline__ u64 mulhi64(u64 a, u64 b) { return __umul64hi(a, b); }

// x * w mod q in [0, 2q) for any x < 2^64, w < q, ws = floor(w 2^64 / q).
__device__ __forceinline__ u64 shoup_lazy(u64 x, u64 w, u64 ws, u64 q)
{
    return x * w - mulhi64(x, ws) * q;
}

__device__ __forceinline__ u64 csub(u64 x, u64 q) { return x >= q ? x - q : x; }

__device__ __forceinline__ u64 shoup(u64 x, u64 w, u64 ws, u64 q)
{
    return csub(shoup_lazy(x, w, ws, q), q);
}


// ---------------------------------------------- exact modular FP64 arithmetic
//
// For q < 2^51 residues and constants are integers held exactly in doubles,
// in balanced form |x| <= q/2.  A product y w mod q is p = y w with its exact
// low part e = fma(y, w, -p), t = rint(p / q) and r = fma(-t, q, p) + e: an
// exact integer congruent to y w, within q + |e| of zero while |p / q| stays
// well below 2^52 (|e| <= ulp(p) / 2).  Sums of such values stay exact below
// 2^53.  No contraction may merge these operations (the split of y w into
// p + e relies on p being the rounded product), hence the per-function
// pragma.

// y w mod q as an exact integer in about (-1.4 q, 1.4 q), for |y w| < 2^104
__device__ __forceinline__ double fmulmod(double y, double w, double q, double qinv)
{
#pragma clang fp contract(off)
    const double p = y * w;
    const double e = __fma_rn(y, w, -p);
    const double t = rint(p * qinv);
    return __fma_rn(-t, q, p) + e;
}

// x - q rint(x / q): balanced representative, |result| <= q/2 + 1
__device__ __forceinline__ double fbal(double x, double q, double qinv)
{
#pragma clang fp contract(off)
    return __fma_rn(-rint(x * qinv), q, x);
}

// Exact conversions between integers below 2^52 and doubles through the
// mantissa of 2^52 + v (one add and one bit operation instead of the generic
// conversion sequences).
constexpr double kTwo52 = 4503599627370496.0;
__device__ __forceinline__ double u2f(u64 v)
{
#pragma clang fp contract(off)
    return __longlong_as_double((long long)(v | 0x4330000000000000ull)) - kTwo52;
}
__device__ __forceinline__ u64 f2u(double y)   // y an integer in [0, 2^52)
{
#pragma clang fp contract(off)
    return (u64)__double_as_longlong(y + kTwo52) & 0xFFFFFFFFFFFFFull;
}

// canonical residue in [0, q) -> balanced double in (-q/2, q/2]
__device__ __forceinline__ double to_bal(u64 v, u64 q, double qd)
{
#pragma clang fp contract(off)
    const double d = u2f(v);
    return v > (q >> 1) ? d - qd : d;
}

// balanced double (any |x| < 2^52.7) -> canonical residue in [0, q)
__device__ __forceinline__ u64 to_canon(double x, double q, double qinv)
{
#pragma clang fp contract(off)
    const u64 v = f2u(fbal(x, q, qinv) + q);   // in [q/2 - 1, 3q/2 + 1]
    const u64 qi = f2u(q);
    return v >= qi ? v - qi : v;
}

__device__ __forceinline__ u32 brev_n(u32 x, u32 log_n) { return __brev(x) >> (32 - log_n); }

// index in the evaluation domain that sigma_g reads for output slot i:
// out[i] = in[brev((g (2 brev(i) + 1) mod 2N - 1) / 2)]
__device__ __forceinline__ u32 galois_src(u32 i, u32 g, u32 log_n)
{
    const u32 two_n_mask = (2u << log_n) - 1;
    const u32 e = (u32)(((u64)g * (2 * brev_n(i, log_n) + 1)) & two_n_mask);
    return brev_n((e - 1) >> 1, log_n);
}

__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q) { return csub(a + b, q); }
__device__ __forceinline__ u64 neg_mod(u64 a, u64 q) { return a ? q - a : 0; }
__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }

// a * b mod q for a, b < q (Barrett with k-bit shifts; remainder < 3q before
// the two corrections).
__device__ __forceinline__ u64 mul_mod(u64 a, u64 b, const ModQ& m)
{
    u64 lo = a * b;
    u64 hi = mulhi64(a, b);
    u32 k = m.k;
    u64 x1 = (hi << (65 - k)) | (lo >> (k - 1));
    u64 plo = x1 * m.mu;
    u64 phi = mulhi64(x1, m.mu);
    u64 q1 = (phi << (63 - k)) | (plo >> (k + 1));
    u64 r = lo - q1 * m.q;
    r = csub(r, m.q);
    return csub(r, m.q);
}

// (hi 2^64 + lo) mod q for any 128-bit value: hi * (2^64 mod q) + lo, each
// reduced with a Shoup product.
__device__ __forceinline__ u64 reduce128(u64 hi, u64 lo, const ModQ& m)
{
    u64 r = shoup_lazy(hi, m.r64, m.r64_s, m.q) + shoup_lazy(lo, 1, m.one_s, m.q);
    r = csub(r, 2 * m.q);
    return csub(r, m.q);
}

// any 64-bit value mod q
__device__ __forceinline__ u64 red64(u64 x, const ModQ& m)
{
    return csub(shoup_lazy(x, 1, m.one_s, m.q), m.q);
}

// 128-bit accumulator helpers
__device__ __forceinline__ void mac128(u64& hi, u64& lo, u64 a, u64 b)
{
    u64 plo = a * b;
    u64 phi = mulhi64(a, b);
    lo += plo;
    hi += phi + (lo < plo ? 1 : 0);
}
#endif

// ----------------------------------------------------------- context

// Device memory owned through shared pointers (ciphertext views into one slab
// keep the slab alive).  Freed stream-ordered on the stream it was allocated
// on, by the allocator that made it.
struct CaptureKeep;

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    void (*free_fn)(void*, void*, void*) = nullptr;
    void* free_user = nullptr;
    std::shared_ptr<DeviceArena> arena;   // built-in allocator (kept alive by its blocks)
    std::shared_ptr<CaptureKeep> cap;     // allocated while a graph was being captured
    ~DevBuf();
};
typedef std::shared_ptr<DevBuf> BufPtr;

// Memory of one captured graph.  While a thread captures (g_capture set),
// every allocation comes from here: a block released during the capture goes
// back to this pool and later allocations of the same capture reuse it -- the
// captured work is one stream-ordered chain, so the reuse is safe on every
// replay -- and no block is recorded in or returned to the context's cache
// while the graph may run.  The blocks go back to the context's allocator
// when the graph and every handle into its memory are gone.
struct CaptureKeep {
    std::shared_ptr<DeviceArena> arena;
    hipStream_t release_stream = nullptr;
    std::mutex mu;
    std::multimap<size_t, void*> free;             // by block size
    std::map<void*, size_t> size;                  // every block it owns
    void* take(size_t bytes);
    void give_back(void* p);
    ~CaptureKeep();
};
extern thread_local std::shared_ptr<CaptureKeep> g_capture;

// Kernel classes the event profiler can bracket.
enum ProfClass : int {
    kProfNtt = 0,       // one forward/inverse NTT call (all its passes); units = limbs
    kProfKsInner,       // key-switch inner product; units = ciphertext x extended limb
    kProfBaseConv,      // fast base conversion; units = output limbs
    kProfLincomb,       // fused MulConst/AddConst accumulation; units = output limbs
    kProfModDown,       // ModDown combine; units = output limbs
    kProfTensor,        // tensor products; units = input limbs
    kProfClasses
};

struct Profiler {
    int cls = -1;
    std::vector<hipEvent_t> ev;   // start/stop pairs
    size_t used = 0;
    u64 units = 0, launches = 0;
    bool overflow = false;
};

// Base-conversion constants for one (input set -> output set) conversion.
struct ConvTable {
    u32 n_in = 0, n_out = 0;
    u64* dev = nullptr;    // device: [n_in] qhat_inv, [n_in] qhat_inv_s, [n_in][n_out] qhat mod t,
                           //         [n_out] (-Q) mod t, then u32 in_mod[n_in], out_mod[n_out]
    size_t words = 0;
    // matrix-core form: balanced base-256 digit words of the same constants,
    // [groups][4][steps][64] (one 64-bit A operand per lane and instruction)
    u64* wt = nullptr;
    u32 steps = 0, groups = 0;
    // FP64 form: [n_out][16][2] balanced constants, then [n_out][2] (t, 1/t);
    // bit i of wide: input modulus i is 2^51 or more
    double* wf = nullptr;
    u32 wide = 0;
    u32 wide_out = 0;   // bit o: target o (o < 31) is 2^51 or more; bit 31: a later one is
    // kernel chosen for this table: -1 not yet timed, 0 vector ALU, 1 MFMA,
    // 2 FP64, 3 FP64 for targets 1.. and the vector ALU for target 0
    std::shared_ptr<std::atomic<int>> choice;
};

}  // namespace vr

struct vr_context {
    int device = 0;
    vr::u32 log_n = 0, n = 0, slots = 0;
    vr::u32 L = 0, K = 0, dnum = 0, alpha = 0;
    double scale = 1.0;
    bool secure = false;
    std::vector<vr::u64> mod;         // q_0..q_L, p_0..p_{K-1}
    std::vector<vr::ModQ> modq;       // host copy
    vr::ModQ* d_modq = nullptr;
    vr::u64* d_tw = nullptr;          // [nmod][N][2] (psi^brev(k), Shoup companion)
    vr::u64* d_itw = nullptr;         // [nmod][N][2] (psi^-brev(k), Shoup companion)
    double* d_twf = nullptr;          // [nmod][N] psi^brev(k) in (-q/2, q/2] (FP64 butterflies)
    double* d_itwf = nullptr;         // [nmod][N] psi^-brev(k) likewise
    double* d_fft_tw = nullptr;       // [N] complex e^{-2 pi i k / 2N}
    // (c, Shoup companion) per modulus: P^-1 mod q_i (Q chain), and for each
    // level l, q_l^-1 mod q_i at [l][i] (i < l): the ModDown and rescale scalings
    ulonglong2* d_pinv_tab = nullptr;  // [nmod]
    ulonglong2* d_rinv_tab = nullptr;  // [L + 1][nmod]: q_l^-1 mod q_i, i < l
    ulonglong2* d_prinv_tab = nullptr; // [L + 1][nmod]: (P q_l)^-1 mod q_i, i < l
    ulonglong2* d_pmod_tab = nullptr;  // [nmod]: P mod q_m (zero on the special primes)
    int* d_gexp = nullptr;            // [S] 5^j mod 2N
    vr::u64 cdt[20];
    std::map<std::pair<int, int>, vr::ConvTable> modup_tables;   // (level, digit)
    // (level, digit, first, end): digit to the extended limbs [first, end)
    std::map<std::array<int, 6>, vr::ConvTable> modup_range_tables;   // {level, digit, e0, e1, e2, e3}
    std::map<int, vr::ConvTable> moddown_tables;                 // level
    std::map<int, vr::ConvTable> moddown_rs_tables;              // level * 1024 + nk: {q_l, P} -> q_<nk
    // device-resident constants of layer calls (weights, term lists), keyed by
    // the call's shape and weight bytes, so repeated calls upload nothing
    std::map<std::string, std::shared_ptr<void>> plans;
    // kernel choices: "base_convert" = 0 autotune, 1 vector ALU, 2 MFMA, 3 FP64;
    // "ntt" = 0 autotune, 1 the fixed default pass plan
    std::map<std::string, int> tuning;
    // NTT pass plans picked by the autotuner, per direction, per pass:
    // {first stage, stages, log groups per workgroup, whole-limb direct, words per
    // thread, stages per round}
    std::vector<std::array<vr::u32, 6>> ntt_plan[2];
    std::mutex mu;
    hipStream_t stream = nullptr;     // used when a call passes stream = NULL
    std::shared_ptr<vr::DeviceArena> arena;
    vr::Profiler prof;
    void* (*alloc_fn)(size_t, void*, void*) = nullptr;
    void (*free_fn)(void*, void*, void*) = nullptr;
    void* alloc_user = nullptr;

    vr::u32 nmod() const { return L + 1 + K; }
    // modulus index of extended limb e at level lv (limbs q_0..q_lv, p_0..)
    vr::u32 ext_mod(vr::u32 e, vr::u32 lv) const { return e <= lv ? e : L + 1 + (e - lv - 1); }
};

struct vr_ciphertext {
    vr_context* ctx = nullptr;
    vr::BufPtr buf;
    vr::u64* data = nullptr;     // [ncomp][level+1][N]
    vr::u32 ncomp = 2, level = 0;
    double scale = 1.0;
};

struct vr_plaintext {
    vr_context* ctx = nullptr;
    vr::BufPtr buf;
    vr::u64* data = nullptr;     // [level+1][N]
    vr::u32 level = 0;
    double scale = 1.0;
    // compact copy when every limb repeats in runs of 2^clog consecutive
    // evaluation-domain words (a polynomial in Z[X^(2^clog)]): [level+1][N >> clog]
    vr::BufPtr cbuf;
    vr::u64* cdata = nullptr;
    vr::u32 clog = 0;
};

struct vr_secret_key {
    vr_context* ctx = nullptr;
    vr::BufPtr buf;
    vr::u64* s = nullptr;        // [L+1+K][N] evaluation domain
};

struct vr_switch_key {
    vr::BufPtr buf;
    vr::u64* data = nullptr;     // [dnum][2][L+1+K][N]
};

struct vr_eval_keys {
    vr_context* ctx = nullptr;
    vr::BufPtr pk_buf;
    vr::u64* pk = nullptr;       // [2][L+1][N]  (b, a)
    vr_switch_key rlk;
    std::map<vr::u32, vr_switch_key> rot;   // Galois element -> key
};

namespace vr {

// ----------------------------------------------------------- memory

BufPtr dev_alloc(vr_context* ctx, size_t bytes, hipStream_t s);
inline u64* as_u64(const BufPtr& b) { return (u64*)b->ptr; }

// Brackets the launches made in its scope with HIP events on `s` when the
// context profiles class `cls` (see vr_profile_start).
struct ProfScope {
    vr_context* ctx;
    hipStream_t s;
    long idx = -1;
    ProfScope(vr_context* c, int cls, hipStream_t st, u64 units) : ctx(c), s(st)
    {
        Profiler& p = c->prof;
        if (p.cls != cls) return;
        if (p.used + 2 > p.ev.size()) {
            p.overflow = true;
            return;
        }
        idx = (long)p.used;
        p.used += 2;
        p.units += units;
        p.launches++;
        (void)hipEventRecord(p.ev[idx], s);
    }
    ~ProfScope()
    {
        if (idx >= 0) (void)hipEventRecord(ctx->prof.ev[idx + 1], s);
    }
};

// ----------------------------------------------------------- launchers

// A set of limbs to transform: limb r (0 <= r < per_poly * n_polys) belongs
// to poly r / per_poly and sits at slot
//   slot = slot0 + (l < skip_at ? l : l + skip_len),   l = r % per_poly,
// i.e. at in + poly * poly_stride + slot * N, with modulus index
//   slot <= level ? slot : L + 1 + slot - level - 1
// (level = -1 puts every slot on the special primes).  With digit_skip the
// skipped range is the Q limbs of digit (poly % beta) (ModUp targets).  The
// output goes to the same place in `out`, or densely to out + r * N when
// out_dense is set.
// Finish of a forward transform (ModDown, rescale): instead of the transform
// y of limb i of poly p = 2 k + j (ciphertext k, component j), store
// (A - y) c (+ B) mod q, with A(p, i) = a + k a_ct + j a_comp + i N,
// out(p, i) = out_j + k out_ct + i N, B(p, i) = add_j + k add_ct + i N
// (component 0 read through sigma_g when add0_g != 1, a null add_j adds
// nothing; B is first multiplied by bmul[modulus of the limb] when bmul is
// set) and (c, floor(c 2^64 / q)) = cmul[modulus of the limb].  The
// limbs of each poly are its first per_poly ones (no skip).  Applied only by
// the whole-limb transform; ntt_forward reports whether it was.
struct NttEpilogue {
    const u64* a = nullptr;        // non-null: the epilogue is requested
    u64 a_ct = 0, a_comp = 0;
    u64* out0 = nullptr;
    u64* out1 = nullptr;
    u64 out_ct = 0;
    const u64* add0 = nullptr;
    const u64* add1 = nullptr;
    u64 add_ct = 0;
    u32 add0_g = 1;
    const ulonglong2* cmul = nullptr;
    const ulonglong2* bmul = nullptr;
};

struct LimbSet {
    u64* in = nullptr;
    u64* out = nullptr;          // may equal in
    u64 poly_stride = 0;         // elements
    u32 per_poly = 0;            // limbs transformed per poly
    u32 n_polys = 0;
    int level = 0;
    u32 slot0 = 0;
    u32 skip_at = 0xffffffffu, skip_len = 0;
    u32 digit_skip = 0, alpha = 0, beta = 0, nq = 0;
    u32 out_dense = 0;
    // slot remap_slot takes modulus remap_mod instead (a compact extended
    // layout that holds q_level right after the kept low limbs)
    u32 remap_slot = 0xffffffffu, remap_mod = 0;
    // forward only: the first pass reads, instead of each limb, the one-limb
    // source it is the fast base conversion of (digits of one modulus): poly
    // p takes limb cv_src + (p / cv_beta) * cv_ct_stride + (p % cv_beta) * N,
    // modulo modulus cv_mod0 + p % cv_beta, centred and reduced to the limb's
    // own modulus on the load
    const u64* cv_src = nullptr;
    u64 cv_ct_stride = 0;
    u32 cv_beta = 1, cv_mod0 = 0;
    NttEpilogue epi;   // forward only, see NttEpilogue
};

// Returns whether ls.epi was applied (false when it is unset or the plan
// for this ring has neither a whole-limb pass nor the compile-time two-pass
// kernels: then the transform is stored).
bool ntt_forward(vr_context* ctx, const LimbSet& ls, hipStream_t s);
void ntt_inverse(vr_context* ctx, const LimbSet& ls, hipStream_t s);

inline LimbSet poly_limbs(u64* in, u64* out, u32 n_polys, u32 per_poly, u64 poly_stride, int level)
{
    LimbSet ls;
    ls.in = in;
    ls.out = out;
    ls.n_polys = n_polys;
    ls.per_poly = per_poly;
    ls.poly_stride = poly_stride;
    ls.level = level;
    return ls;
}

}  // namespace vr
