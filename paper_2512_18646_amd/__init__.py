"""MI355X (gfx950) implementation of the column-wise encrypted-inference path
of Volley Revolver (Inference++): RNS-CKKS ciphertext arithmetic in HIP
kernels behind the C ABI of include/vr.h, with this thin Python binding.

    from paper_2512_18646_amd import vr
    ctx = vr.Context(14, [60] + [40] * 7, [60], 8, 40.0)
"""
__all__ = ["vr", "build"]
