"""The oracle's pins catch plausible mistakes: each case plants one mistake in a
copy of the oracle's source (a dropped factor, a flipped rule, a wrong index),
builds it with gcc on the CPU, and runs the pin that must fail for it.  The
oracle itself is never altered; the copies live in the test's temporary folder."""
import os

import pytest

from tests import test_oracle_healpix as hp
from tests import test_oracle_physics as phys

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "art_oracle.c")

MUTATIONS = [
    # Sec. 2.1 tau_max with several bins: destroy once ANY bin is thick
    ("any_bin_termination",
     """            int all_thick = 1;
            for (int q = 0; q < nb; ++q) {
                tau[q] += kap[q] * dr;
                if (!(tau[q] > P->tau_term)) all_thick = 0;
            }""",
     """            int all_thick = 0;
            for (int q = 0; q < nb; ++q) {
                tau[q] += kap[q] * dr;
                if (tau[q] > P->tau_term) all_thick = 1;
            }""",
     phys.test_termination_every_bin),
    # Eq. e:Erad: J deposited without the (1 - e^-x)/x factor
    ("J_without_phi",
     "Jw[q * N + g->cell] += Lin * g->dr * orc_phi(g->dtau[q]);",
     "Jw[q * N + g->cell] += Lin * g->dr;",
     phys.test_estimator_consistency),
    # Eq. e:Frad: momentum deposited against the ray direction
    ("force_sign",
     "force[0 * N + g->cell] += n[0] * dLsum;",
     "force[0 * N + g->cell] -= n[0] * dLsum;",
     phys.test_momentum_bookkeeping),
    # Sec. 2.1: packets not divided among the four children
    ("packet_not_divided",
     "for (int q = 0; q < nb; ++q) Lnom[q] = Ls[q] / (12.0 * ldexp(1.0, 2 * l));\n            if (st)",
     "for (int q = 0; q < nb; ++q) Lnom[q] = Ls[q] / (12.0 * ldexp(1.0, 2 * P->level0));\n            if (st)",
     lambda O: phys.test_photon_conservation(O, 3.0)),
    # Sec. 2.1: children start at their own split radius instead of the parent's
    ("child_start_radius",
     "const double r_a = (l == P->level0) ? 0.0 : orc_r_max(P->phi_c, l - 1);\n            const double r_split = (l < P->level_max) ? orc_r_max(P->phi_c, l) : INFINITY;\n            const double d_exit = orc_exit_distance(P, xs, n);\n            /* packet",
     "const double r_a = (l == P->level0) ? 0.0 : orc_r_max(P->phi_c, l);\n            const double r_split = (l < P->level_max) ? orc_r_max(P->phi_c, l) : INFINITY;\n            const double d_exit = orc_exit_distance(P, xs, n);\n            /* packet",
     phys.test_uniform_medium_escape_closed_form),
    # adjoint: the loss carried downstream of a segment left out of dL/dkappa
    ("adjoint_without_downstream",
     """            const double dk = aq * Lin * g->dr * g->dr * orc_dphi(x) + beta * Lin * g->dr * e
                              - g->dr * Gq[q];""",
     """            const double dk = aq * Lin * g->dr * g->dr * orc_dphi(x) + beta * Lin * g->dr * e;""",
     phys.test_adjoint_vs_central_differences),
    # Sec. 2.3 opacities: the non-ionizing bin absorbed by the gas too
    ("gas_in_nonionizing_bin",
     "    return nH[c] * P->s_d;\n}",
     "    return nH[c] * (xn[c] * P->s_H + P->s_d);\n}",
     phys.test_termination_every_bin),
    # Sec. 2.1: an escaping packet counted at its launch luminosity, not attenuated
    ("escaped_unattenuated",
     "const double Lleft = Lnom[q] * exp(-tau[q]);",
     "const double Lleft = Lnom[q];",
     lambda O: phys.test_photon_conservation(O, 3.0)),
    # Sec. 2.2 destroy counter: an ended ray weighted as one of the level below
    ("destroy_weight",
     "st->destroy += (uint64_t)1 << (2 * (P->level_max - l));",
     "st->destroy += (uint64_t)1 << (2 * (P->level_max - l - 1));",
     lambda O: phys.test_destroy_counter_total(O, 0)),
    # Eq. e:photrate2: the rate without the neutral fraction (n_H instead of n_HI)
    ("rate_without_xn",
     "for (int64_t c = 0; c < N; ++c) rate[c] = P->s_H * xn[c] * nH[c] * Jw[c];",
     "for (int64_t c = 0; c < N; ++c) rate[c] = P->s_H * nH[c] * Jw[c];",
     phys.test_rate_counts_every_gas_absorption),
    # adjoint chain rule: d kappa_i / d x_n taken as n_H (s_H + s_d)
    ("adjoint_chain_xn",
     "g_xn[c] = gk[c] * nH[c] * P->s_H + w[c] * P->s_H * nH[c] * J[c];",
     "g_xn[c] = gk[c] * nH[c] * (P->s_H + P->s_d) + w[c] * P->s_H * nH[c] * J[c];",
     phys.test_adjoint_vs_central_differences),
    # Sec. 2.1: the split radius with pi m_ray replaced by 2 pi m_ray
    ("split_radius",
     "return sqrt(3.0 / (M_PI * phi_c)) * ldexp(1.0, level);",
     "return sqrt(3.0 / (2.0 * M_PI * phi_c)) * ldexp(1.0, level);",
     phys.test_tree_closed_form_workload1),
    # HEALPix (Gorski et al. 2005): pixel centres shifted by half a pixel in phi
    ("healpix_phi_shift",
     "*phi = (M_PI / (2.0 * (double)nr)) * ((double)j - 0.5 * (double)(2 - s));",
     "*phi = (M_PI / (2.0 * (double)nr)) * ((double)j - 0.5 * (double)(1 - s));",
     lambda O: hp.test_nested_centres_equal_ring_centres(O, 2)),
    # Eq. e:Erad: the small-optical-depth series of (1 - e^-x)/x with a wrong sign
    ("phi_series_sign",
     "if (fabs(x) < 1e-5) return 1.0 - x / 2.0 + x * x / 6.0;",
     "if (fabs(x) < 1e-5) return 1.0 + x / 2.0 + x * x / 6.0;",
     phys.test_estimator_in_the_optically_thin_limit),
    # Sec. 2.2 Step 1: seeds injected face by face instead of interleaved
    ("seed_order_by_face",
     "r.pix = (k % 12) * per_face + k / 12;",
     "r.pix = k;",
     phys.test_seed_order_step1),
]


@pytest.mark.parametrize("name,old,new,pin", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_mutation(tmp_path, name, old, new, pin):
    from oracle import oracle as O
    src = open(SRC).read()
    assert src.count(old) == 1, f"{name}: the snippet to alter is not in the oracle (once)"
    bad = tmp_path / f"oracle_{name}.c"
    bad.write_text(src.replace(old, new))
    lib = O.compile_library(str(bad), str(tmp_path / f"liboracle_{name}.so"))
    with O.using_library(lib):
        with pytest.raises(AssertionError):
            pin(O)
    # and the pin passes on the oracle itself
    pin(O)
