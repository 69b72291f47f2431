"""Flop and algorithmic-byte conventions (host-side bookkeeping only).

Flops follow the per-site count of Table 1 (Sec. 2): the hopping term H costs
1320 flop per output site -- for each of the 8 directions a 12-flop spin
projection and two 66-flop SU(3) matrix-vector products, plus 7 x 24 flop to
accumulate the 8 reconstructed contributions -- and the full D = 1 - kappa*H adds
48 flop (scale and add of 24 reals) for 1368 flop per site.

Algorithmic bytes count each datum the kernel must touch exactly once (the
"ideal" reuse of the paragraph after Table 1):
  parity hop, per output site : 8 links x 18 reals + 24 input reals + 24 output reals
                                (192 reals: FP64 1536 B, FP32 768 B; FP16 spinors carry a
                                4-byte FP32 scale per site);
  full D, per site             : 4 links x 18 + 24 in + 24 out = 120 reals (960 B in FP64).
Table 1's own "no reuse" float figure, 1536 B per site of D, counts 8 links, 8
neighbour spinors, the site spinor and the output.
"""

HOP_FLOPS_PER_SITE = 8 * (12 + 2 * 66) + 7 * 24  # 1320
DIAG_FLOPS_PER_SITE = 48
FULL_D_FLOPS_PER_SITE = HOP_FLOPS_PER_SITE + DIAG_FLOPS_PER_SITE  # 1368
# clover matrix (Sec. 2.1.2): two Hermitian 6x6 block mat-vecs, each 36 complex products
# (6 flop) and 30 complex additions (2 flop), on top of the Wilson count
CLOVER_TERM_FLOPS_PER_SITE = 2 * (36 * 6 + 30 * 2)  # 552
CLOVER_FLOPS_PER_SITE = FULL_D_FLOPS_PER_SITE + CLOVER_TERM_FLOPS_PER_SITE + 24  # 1944 (Table 1)

REAL_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2}


def spinor_site_bytes(prec):
    """Bytes of one site's spinor in storage precision (FP16 adds the FP32 per-site scale)."""
    return 24 * REAL_BYTES[prec] + (4 if prec == "fp16" else 0)


def link_bytes(prec):
    return 18 * REAL_BYTES[prec]


def hop_bytes_per_site(spinor_prec, link_prec=None):
    """Algorithmic bytes of the parity hop per output site."""
    link_prec = link_prec or spinor_prec
    return 8 * link_bytes(link_prec) + 2 * spinor_site_bytes(spinor_prec)


def clover_term_bytes(prec):
    """F(x) per site: two Hermitian 6x6 blocks = 72 reals."""
    return 72 * REAL_BYTES[prec]


def clover_full_bytes_per_site(prec):
    """Algorithmic bytes of D_clov per site with ideal reuse: the Wilson count plus F."""
    return full_d_bytes_per_site(prec) + clover_term_bytes(prec)


def full_d_bytes_per_site(prec):
    """Algorithmic bytes of D = 1 - kappa*H per site with ideal reuse."""
    return 4 * link_bytes(prec) + 2 * spinor_site_bytes(prec)


def table1_no_reuse_bytes_per_site(prec="fp32"):
    """Table 1's float count: 8 links + 8 neighbour spinors + the site spinor + the output."""
    return 8 * link_bytes(prec) + 8 * spinor_site_bytes(prec) + 2 * spinor_site_bytes(prec)


def bicgstab_iter_bytes_per_even_site(prec="fp64"):
    """Fused even-odd BiCGStab iteration per even site (reals): 4 hops + xpay/dot
    epilogues + 3 vector kernels = 1176 reals."""
    reals = (96 + 192 + 240 + 72 + 192 + 216 + 168)
    return reals * REAL_BYTES[prec]


# Peak figures of the MI355X used for roofline fractions (published spec values).
MI355X_HBM_GBS = 8000.0
MI355X_FP64_VECTOR_TFLOPS = 78.6
MI355X_FP32_VECTOR_TFLOPS = 157.3
