"""The benchmark's algorithmic byte model (bench.pass_bytes_per_point and
bench.all_fields_bytes_per_point), which every roofline fraction it reports
divides by: per pass and in total against the pass table (one read and one
write of each field a pass touches; a half spectrum holds c bytes per grid
point and field, c = 4 mixed and 8 FP64; eight stored FMT fields on the x
side of the y passes; densities in and mu, exp(-mu) out in FP64) and the
closed forms 60 S + 28.8 F (mixed) and 60 S + 32 F with all ten fields."""
import pytest

import bench

MIXED, FP64 = 1, 0


def test_pass_table_mixed_three_species():
    got = bench.pass_bytes_per_point(3, MIXED)
    want = {"z_fwd_rho": 36, "y_fwd_rho": 24, "x_fwd_weights": 44, "y_inv_n": 72, "z_deriv": 80,
            "y_fwd_dphi": 72, "x_back_pairs": 56, "y_inv_mu": 24, "z_inv_final": 60}
    assert got == want
    assert sum(got.values()) == 468


def test_pass_table_fp64_three_species():
    got = bench.pass_bytes_per_point(3, FP64)
    assert got == {"z_fwd_rho": 48, "y_fwd_rho": 48, "x_fwd_weights": 88, "y_inv_n": 144, "z_deriv": 160,
                   "y_fwd_dphi": 144, "x_back_pairs": 112, "y_inv_mu": 48, "z_inv_final": 72}
    assert sum(got.values()) == 864


@pytest.mark.parametrize("S", [1, 2, 3, 4, 8])
def test_closed_forms(S):
    # mixed: 60 S + 28.8 F with F = 10 (8 stored fields on the x side)
    assert sum(bench.pass_bytes_per_point(S, MIXED).values()) == pytest.approx(60 * S + 28.8 * 10)
    assert sum(bench.all_fields_bytes_per_point(S, MIXED).values()) == 60 * S + 32 * 10
    assert sum(bench.all_fields_bytes_per_point(S, FP64).values()) == 96 * S + 64 * 10


def test_without_slotboom_output():
    # without exp(-mu) the last pass writes only mu (8 bytes per point and species)
    full = bench.pass_bytes_per_point(3, MIXED)
    bare = bench.pass_bytes_per_point(3, MIXED, slot=False)
    assert full["z_inv_final"] - bare["z_inv_final"] == 8 * 3
    assert {k: v for k, v in full.items() if k != "z_inv_final"} == {k: v for k, v in bare.items() if k != "z_inv_final"}


def _oracle_offsets(r, k, cubic):
    """Distinct grid offsets with a nonzero interpolation weight over the
    nodes of the oracle's rule (its node directions and per-axis weights)."""
    import math
    import numpy as np
    import oracle.sphere_quad as sq
    theta, _, phi, _ = sq.sphere_rule(k)
    seen = set()
    for th in theta:
        for ph in phi:
            p = r * np.array([math.cos(th) * math.sin(ph), math.sin(th) * math.sin(ph), math.cos(ph)])
            base = np.floor(p).astype(np.int64)
            ax = [sq.axis_weights(p[a] - base[a], cubic) for a in range(3)]
            for ox, wx in zip(*ax[0]):
                for oy, wy in zip(*ax[1]):
                    for oz, wz in zip(*ax[2]):
                        if float(wx * wy * wz) != 0.0:
                            seen.add((int(base[0] + ox), int(base[1] + oy), int(base[2] + oz)))
    return len(seen)


@pytest.mark.parametrize("cubic", [False, True])
@pytest.mark.parametrize("r,k", [(1.5, 8), (3.0, 8), (4.0, 8), (3.0, 4), (2.0, 16)])
def test_sphere_stencil_count_matches_the_oracle_rule(r, k, cubic):
    """The sphere workload's flop count rests on the number of distinct
    stencil offsets; counted from the oracle's rule it must agree."""
    assert bench.sphere_stencil_size(r, k, cubic) == _oracle_offsets(r, k, cubic)
