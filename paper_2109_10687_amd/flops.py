"""Flop and byte accounting for the Clover-Wilson operator and its solvers.

Per-site flop counts (the convention the paper's theoretical FLOP columns use,
Sec. 5, Tables 2 and 3):

* one hop (one direction, one sign): spin projection to a half-spinor (12),
  two SU(3) matrix-vector products (2 x 66) and the accumulation back into the
  four-spinor (24): 168 flop for x, y, z.  gamma_4 is diagonal, so the t hop
  needs no projection adds: 156.
* clover multiply: two 6x6 Hermitian blocks (2 x 276) plus the combine (48): 600.
* one full D or A apply: 2 x (3 x 168 + 156) + 600 = 1920 flop per site.

The per-rank totals of Tables 2 and 3 follow from these counts with the SAP loop
count 4 and Jacobi count 2; the fitted per-site vector-operation term and the
per-rank scalar term of Table 2 are the only constants not derived here.
"""
from math import prod

HOP_FLOPS = (168, 168, 168, 156)  # per hop in x, y, z, t
CLOVER_FLOPS = 600
FULL_HOP_FLOPS = 2 * sum(HOP_FLOPS)  # 1320
DIRAC_FLOPS_PER_SITE = FULL_HOP_FLOPS + CLOVER_FLOPS  # 1920

# algorithmic bytes per site of one full apply: input spinor, output spinor,
# four links (each link is used by two sites and counted once), clover block
SPINOR_REALS = 24
LINK_REALS = 18
LINK_REALS_COMPRESSED = 12
CLOVER_REALS = 72


def dirac_bytes_per_site(real_bytes, link_reals=LINK_REALS, spinor_scale_bytes=0):
    """Bytes one apply must move per site with the given real width."""
    spinor = SPINOR_REALS * real_bytes + spinor_scale_bytes
    return 2 * spinor + 4 * link_reals * real_bytes + CLOVER_REALS * real_bytes


def in_domain_hop_flops(domain):
    """Hop flops per site that stay inside a Schwarz domain of extent `domain` (x, y, z, t)."""
    return sum(2 * (d - 1) / d * c for d, c in zip(domain, HOP_FLOPS))


def surface_fraction(domain):
    """Fraction of domain sites with at least one neighbour outside the domain."""
    interior = prod(max(d - 2, 0) for d in domain)
    return 1.0 - interior / prod(domain)


# constants of the paper's Table 2 accounting that the per-site counts above do
# not fix: vector operations per site per BiCGStab iteration, and a per-rank
# scalar term for the whole 500-iteration run
TABLE2_VECTOR_FLOPS = 2400
TABLE2_SCALAR_FLOPS = 21000


def paper_domain(rank_dims):
    """Each rank holds two SAP domains, one per colour, split along x (Sec. 3)."""
    x, y, z, t = rank_dims
    return (x // 2, y, z, t)


def table3_flop(rank_dims, n_sap=4, iters=500):
    """FLOP of the A_EE/A_OO regions: 2 (n_sap + 1) in-domain applies per iteration."""
    dom = paper_domain(rank_dims)
    per_site = 2 * (n_sap + 1) * (in_domain_hop_flops(dom) + CLOVER_FLOPS)
    return iters * prod(rank_dims) * per_site


def table2_flop(rank_dims, n_sap=4, n_jac=2, iters=500):
    """FLOP of the whole SAP-BiCGStab run: per block apply pass the in-domain apply,
    n_jac Jacobi applies and the cross-domain apply on surface sites."""
    dom = paper_domain(rank_dims)
    fin = in_domain_hop_flops(dom)
    surf = surface_fraction(dom)
    ddd_in = fin + CLOVER_FLOPS
    jinv = n_jac * (fin + CLOVER_FLOPS)
    ddd_out = (FULL_HOP_FLOPS - fin) + CLOVER_FLOPS * surf
    per_site = 2 * (n_sap + 1) * (ddd_in + jinv + ddd_out) + TABLE2_VECTOR_FLOPS
    return iters * prod(rank_dims) * per_site + TABLE2_SCALAR_FLOPS


def sap_block_applies(n_sap, n_jac):
    """Full-lattice-equivalent in-block applies in one application of A M_SAP:
    (n_sap + 1) passes over both colours, each n_jac Jacobi applies plus one."""
    return (n_sap + 1) * (n_jac + 1)
