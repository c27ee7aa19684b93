"""Workload constants of the synthetic configurations.

C0  plain VEGAS on a d=4 normalised Gaussian product (FP64 integrand).
C1  log-bicubic PDF interpolation alone on a synthetic 11-flavour grid.
C2  LO pp -> t tbar at sqrt(s) = 13 TeV, 3-d (tau, y, cos theta*) integrand.
C3  64 independent integrals of uneven dimension and sample count, batched.
C4  coupling-flow proposal trained on VEGAS samples, compared with VEGAS.
C5  LO Drell-Yan (gamma*/Z -> l+ l-) at sqrt(s) = 13 TeV on the C2 path.
C6  LO s-channel single top (u dbar -> t bbar) at sqrt(s) = 8 TeV on the C2 path.
C7  multi-member PDF evaluation: N_rep members of a synthetic set, all 11
    flavours at 2415 x points of a FastKernel-type grid.
"""

# Flavour order of every PDF array: PDG ids -5..-1, gluon (21), 1..5.
FLAVOURS = (-5, -4, -3, -2, -1, 21, 1, 2, 3, 4, 5)

C0 = dict(
    name="vegas-gauss4-f64",
    dim=4, n_bins=50, alpha=1.5, iterations=10, n_per_iter=100_000,
    seed=0, stream=0,
    centre=0.5, sigma=0.1,
    # Large-sample variant used to fill the chip (1e5 samples only occupy a
    # fraction of 256 CUs for a few microseconds).
    n_per_iter_large=1_000_000_000,
)

C1 = dict(
    name="pdf-logbicubic-11flav",
    n_x=196, x_min=1e-9, x_max=1.0,
    # Q subgrid boundaries in GeV: nodes start at 1 GeV, thresholds at
    # 1.3 (charm) and 4.75 (bottom), top at 1e5.  4 + 12 + 34 = 50 log-Q^2
    # nodes, the threshold nodes duplicated in both neighbouring subgrids.
    q_edges=(1.0, 1.3, 4.75, 1.0e5), nq_per_sub=(4, 12, 34),
    lambda_qcd=0.2, q0=1.0,
    grid_seed=1,
    n_queries=100_000_000,
    query_q_min=1.65, query_q_max=1.0e5,
    query_seed=0xC1,
)

C2 = dict(
    name="ttbar-lo-13tev",
    dim=3, n_bins=50, alpha=1.5, iterations=10, n_per_iter=10_000_000,
    seed=2, stream=0,
    sqrt_s=13000.0, m_top=173.0, alpha_s=0.118,
    # GeV^-2 -> pb conversion, (hbar c)^2 = 0.3893793721 mb GeV^2.
    gev2_to_pb=3.893793721e8,
)

C3 = dict(
    name="batched-64",
    n_integrals=64, dim_min=2, dim_max=12,
    n_min=10_000, n_max=10_000_000,
    n_bins=50, alpha=1.5, iterations=10,
    seed=3,
)

C4 = dict(
    name="flow-vs-vegas",
    n_layers=4, n_bins=32, hidden=64,
    batch=100_000, steps=200, lr=1e-3,
    beta1=0.9, beta2=0.999, eps=1e-8,
    seed=4,
    gauss_dim=8, gauss_sigma=0.05, gauss_centre=0.5,
)

# LO Drell-Yan, q qbar -> gamma*/Z -> l+ l- (massless leptons), on the same
# fused path as C2: 3-d (tau, y, cos theta*) over a dilepton-mass window,
# PDFs at the fixed scale mu = M_Z.  Electroweak inputs: fixed alpha(M_Z),
# on-shell sin^2 theta_W, Z mass and width.
C5 = dict(
    name="drell-yan-lo-13tev",
    dim=3, n_bins=50, alpha=1.5, iterations=10, n_per_iter=10_000_000,
    seed=5, stream=0,
    sqrt_s=13000.0, m_lo=60.0, m_hi=120.0,
    m_z=91.1876, gamma_z=2.4952, sw2=0.2312, alpha_em=1.0 / 128.0,
    gev2_to_pb=3.893793721e8,
)

# LO single top (s channel): u dbar, c sbar -> W* -> t bbar, the thesis's own
# LO example (pp -> t + 1 jet at the LHC Run 1 energy, m_t = 173.2 GeV), on
# the same fused path: 3-d (tau, y, cos theta*), PDFs at mu = m_t, diagonal
# CKM matrix, fixed alpha and sin^2 theta_W.
C6 = dict(
    name="single-top-s-lo-8tev",
    dim=3, n_bins=50, alpha=1.5, iterations=10, n_per_iter=10_000_000,
    seed=6, stream=0,
    sqrt_s=8000.0, m_top=173.2, m_w=80.385, gamma_w=2.085, sw2=0.2312, alpha_em=1.0 / 128.0,
    gev2_to_pb=3.893793721e8,
)

# Multi-member evaluation (the thesis's FastKernel-type benchmark: 11
# flavours of N_rep members at 2415 x points).  The thesis gives neither the
# scale nor the x distribution: the points sit at Q0 = 1.65 GeV (a typical
# fitting scale, inside the charm subgrid of C1), x log-spaced in [1e-7, 0.9].
# Members: C1's grid times a smooth seeded factor 1 + eps (a + b ln x / ln 1e-9)
# per member and flavour (a, b standard normal), so zero nodes stay zero.
C7 = dict(
    name="pdf-members-fk-2415",
    n_points=2415, q=1.65, x_lo=1e-7, x_hi=0.9,
    n_rep=(10, 50, 100, 200, 300, 400), eps=0.05, seed=7,
)
