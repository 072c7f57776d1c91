// CKKS encoding and decoding on the GPU (FP64).
//
// Encode: slot j sits at the root psi^(g_j), g_j = 5^j mod 2N; the real slot
// vector z gives the integer polynomial
//     m_t = RHA((2 scale / N) Re sum_j z_j exp(-i pi g_j t / N)),
// i.e. the real part of a 2N-point DFT of the vector holding z_j at index g_j.
// Decode reads limb q_0 (centred) and takes z_j = Re DFT(c)[g_j] / scale.
// The DFT is a radix-2 Stockham FFT (self-sorting, one launch per stage,
// batched over vectors); twiddles e^{-2 pi i k / 2N} come from a host table
// computed in long double.
#include "vr_ops.h"

namespace vr {

namespace {

constexpr int kThreads = 256;

__global__ void k_scatter_slots(double2* w, const double* x, u32 n, u64 x_stride, const int* gexp,
                                u32 m_points)
{
    u32 j = blockIdx.x * kThreads + threadIdx.x;
    u32 v = blockIdx.y;
    if (j >= n) return;
    w[(size_t)v * m_points + gexp[j]] = make_double2(x[(size_t)v * x_stride + j], 0.0);
}

__global__ void k_fft_stage(const double2* in, double2* out, u32 m_points, u32 log_ns,
                            const double2* tw)
{
    u32 j = blockIdx.x * kThreads + threadIdx.x;
    u32 half = m_points >> 1;
    if (j >= half) return;
    size_t base = (size_t)blockIdx.y * m_points;
    u32 ns = 1u << log_ns;
    u32 k = j & (ns - 1);
    double2 w = tw[(size_t)k * (m_points >> (log_ns + 1))];
    double2 a0 = in[base + j];
    double2 b = in[base + j + half];
    double2 a1 = make_double2(b.x * w.x - b.y * w.y, b.x * w.y + b.y * w.x);
    u32 d = ((j >> log_ns) << (log_ns + 1)) + k;
    out[base + d] = make_double2(a0.x + a1.x, a0.y + a1.y);
    out[base + d + ns] = make_double2(a0.x - a1.x, a0.y - a1.y);
}

// m_t = RHA(c * Re F[t]) reduced into nl limbs
// sub_mask != 0: coefficients t with t & sub_mask off the subring are zero
__global__ void k_round_to_limbs(const double2* F, u32 m_points, double c, u64* limbs, u32 nl,
                                 u64 limbs_stride, u32 log_n, const ModQ* mq, int* overflow, u32 sub_mask)
{
    u32 t = blockIdx.x * kThreads + threadIdx.x;
    u32 n = 1u << log_n;
    if (t >= n) return;
    u32 v = blockIdx.y;
    double x = (t & sub_mask) ? 0.0 : round(c * F[(size_t)v * m_points + t].x);
    if (!(fabs(x) < 4611686018427387904.0)) {   // 2^62
        *overflow = 1;
        x = 0.0;
    }
    i64 mi = (i64)x;
    u64* out = limbs + (size_t)v * limbs_stride;
    for (u32 l = 0; l < nl; l++) {
        const ModQ m = mq[l];
        u64 r = mi >= 0 ? red64((u64)mi, m) : neg_mod(red64((u64)(-mi), m), m.q);
        out[(size_t)l * n + t] = r;
    }
}

__global__ void k_centre_limb0(double2* w, const u64* c, u32 n, u64 q0)
{
    u32 t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= 2 * n) return;
    double v = 0.0;
    if (t < n) {
        u64 x = c[t];
        v = x > (q0 >> 1) ? -(double)(q0 - x) : (double)x;
    }
    w[t] = make_double2(v, 0.0);
}

__global__ void k_gather_slots(double* out, const double2* F, u32 n, const int* gexp, double scale)
{
    u32 j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= n) return;
    out[j] = F[gexp[j]].x / scale;
}

// forward DFT of n_vec vectors of m points; returns the buffer holding the result
double2* fft(vr_context* ctx, double2* a, double2* b, u32 n_vec, hipStream_t s)
{
    u32 m_points = 2 * ctx->n;
    u32 log_m = ctx->log_n + 1;
    dim3 grid((m_points / 2 + kThreads - 1) / kThreads, n_vec);
    for (u32 st = 0; st < log_m; st++) {
        hipLaunchKernelGGL(k_fft_stage, grid, dim3(kThreads), 0, s, a, b, m_points, st,
                           (const double2*)ctx->d_fft_tw);
        VR_CHECK_LAUNCH();
        std::swap(a, b);
    }
    return a;
}

}  // namespace

void encode_to_limbs(vr_context* ctx, const double* x_dev, u32 n, u32 n_vec, u64 vec_stride_x,
                     double scale, u64* limbs, u32 nl, u64 limbs_stride, hipStream_t s, u32 sub_log)
{
    u32 m_points = 2 * ctx->n;
    size_t bytes = (size_t)n_vec * m_points * sizeof(double2);
    BufPtr wa = dev_alloc(ctx, bytes, s), wb = dev_alloc(ctx, bytes, s);
    BufPtr flag = dev_alloc(ctx, sizeof(int), s);
    VR_HIP(hipMemsetAsync(wa->ptr, 0, bytes, s));
    VR_HIP(hipMemsetAsync(flag->ptr, 0, sizeof(int), s));
    if (n > 0) {
        dim3 g1((n + kThreads - 1) / kThreads, n_vec);
        hipLaunchKernelGGL(k_scatter_slots, g1, dim3(kThreads), 0, s, (double2*)wa->ptr, x_dev, n,
                           vec_stride_x, ctx->d_gexp, m_points);
        VR_CHECK_LAUNCH();
    }
    double2* F = fft(ctx, (double2*)wa->ptr, (double2*)wb->ptr, n_vec, s);
    dim3 g2((ctx->n + kThreads - 1) / kThreads, n_vec);
    hipLaunchKernelGGL(k_round_to_limbs, g2, dim3(kThreads), 0, s, F, m_points,
                       2.0 * scale / (double)ctx->n, limbs, nl, limbs_stride, ctx->log_n,
                       ctx->d_modq, (int*)flag->ptr, (1u << sub_log) - 1);
    VR_CHECK_LAUNCH();
    int ovf = 0;
    VR_HIP(hipMemcpyAsync(&ovf, flag->ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    VR_HIP(hipStreamSynchronize(s));
    if (ovf) throw Error(VR_EINVAL, "encode: coefficient magnitude >= 2^62 (scale too large)");
}

void decode_from_limb0(vr_context* ctx, const u64* coef0, double scale, double* out_dev, u32 n,
                       hipStream_t s)
{
    u32 m_points = 2 * ctx->n;
    size_t bytes = (size_t)m_points * sizeof(double2);
    BufPtr wa = dev_alloc(ctx, bytes, s), wb = dev_alloc(ctx, bytes, s);
    hipLaunchKernelGGL(k_centre_limb0, dim3((m_points + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       s, (double2*)wa->ptr, coef0, ctx->n, ctx->mod[0]);
    VR_CHECK_LAUNCH();
    double2* F = fft(ctx, (double2*)wa->ptr, (double2*)wb->ptr, 1, s);
    hipLaunchKernelGGL(k_gather_slots, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                       out_dev, F, n, ctx->d_gexp, scale);
    VR_CHECK_LAUNCH();
}

}  // namespace vr
