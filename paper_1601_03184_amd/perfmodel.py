"""Byte and flop model of the setup kernels (algorithmic counts, not measurements).

The paper's argument (Sec. 6) compares the memory traffic a complex mat-vec needs
per unit of arithmetic with that of a mat-mat over N right-hand sides: the matrix
element stays on chip for all N.  The same argument, redone for the Wilson-clover
stencil on MI355X, gives the algorithmic bytes per site-RHS used for roofline
fractions.  Flop counts: the stencil is 1320 (8 hops with spin projection) + 504
(two Hermitian 6x6 clover blocks) + 24 (combine) = 1848 flop per site and RHS;
a minimal-residual step adds two inner products and two complex axpys (336).
"""

STENCIL_FLOP = 1848          # per site and RHS, one application of D
MR_EXTRA_FLOP = 336          # <q,q>, <q,rho>, e += a rho, rho -= a q (12 complex each)
RESIDUAL_EXTRA_FLOP = 24     # r = b - D x
LINK_REALS = 18              # one SU(3) matrix
CLOVER_REALS = 72            # two Hermitian 6x6 blocks (6 real diagonal + 15 complex each)
SPINOR_REALS = 24            # 4 spins x 3 colours, complex


def paper_required_bytes_per_cycle(K, M, n_rhs=None, lanes=16, complex_bytes=8):
    """Sec. 6: bytes per cycle per core a complex (M x K) product needs to avoid stalls.

    One complex FMA is 4 real FMAs; a core does `lanes` real FMAs per cycle.  Mat-vec
    (n_rhs None): (2M + MK + K) complex numbers per 4MK/lanes cycles.  Mat-mat with
    n_rhs columns: the matrix is read once for all of them."""
    cycles = 4.0 * M * K / lanes
    if n_rhs is None:
        return (2 * M + M * K + K) * complex_bytes / cycles
    return (2 * M * n_rhs + M * K + K * n_rhs) * complex_bytes / (cycles * n_rhs)


def paper_required_gbs(bytes_per_cycle, cores, clock_ghz):
    return bytes_per_cycle * cores * clock_ghz


def coarse_fine_memory_ratio(n_tv, domain_volume):
    """Sec. 7: coarse vector (2 N_tv complex per domain) over fine vector (12 complex per site)."""
    return 2.0 * n_tv / (12.0 * domain_volume)


def setup_memory_factor(fine_mrhs, coarse_mrhs, fine_srhs, coarse_srhs, ratio):
    return (fine_mrhs + coarse_mrhs * ratio) / (fine_srhs + coarse_srhs * ratio)


def stencil_bytes_per_site_rhs(n_rhs, store_bytes, field_bytes):
    """dirac_apply_mrhs: links (4 forward) + clover read once per site for all n_rhs RHS,
    spinor read once and written once per site and RHS."""
    return (4 * LINK_REALS + CLOVER_REALS) * field_bytes / n_rhs + 2 * SPINOR_REALS * store_bytes


def sap_half_sweep_bytes(V_colour, n_rhs, store_bytes, field_bytes, halo_sites, first):
    """Algorithmic HBM bytes of one SAP half-sweep launch over the blocks of one colour.

    V_colour sites of that colour's blocks, n_rhs RHS.  Reads b and x on the blocks,
    x on the halo (sites outside the blocks that the residual reaches), the fields once
    per site (links of the block's sites and of the halo's backward links, clover),
    writes x.  The first half-sweep starts from x = 0: no x read, no halo."""
    s = SPINOR_REALS * store_bytes
    fields = V_colour * (4 * LINK_REALS + CLOVER_REALS) * field_bytes
    if first:
        vec = V_colour * n_rhs * (s + s)          # read b, write x
    else:
        vec = V_colour * n_rhs * (3 * s) + halo_sites * n_rhs * s   # b, x, write x; halo x
    return fields + vec


def sap_half_sweep_flop(V_colour, n_rhs, n_mr, first, block_hops_fraction):
    """Flops of one SAP half-sweep: residual (skipped from x = 0) + n_mr MR steps on the
    block operator, whose hops are block_hops_fraction of the full stencil's hops."""
    hop, rest = 1320.0, STENCIL_FLOP - 1320.0
    block_stencil = rest + hop * block_hops_fraction
    per = n_mr * (block_stencil + MR_EXTRA_FLOP) + (0 if first else STENCIL_FLOP + RESIDUAL_EXTRA_FLOP)
    return V_colour * n_rhs * per
