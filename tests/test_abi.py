"""Host-side checks of the C ABI: the library loads and exports every function
include/pnp_cdft.h declares, and the host-only entry points answer without a
device (no compute calls here)."""
import ctypes
import os
import re

import pytest

import paper_1407_0674_amd as pkg
from paper_1407_0674_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pnp_cdft.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pnp_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_expected_calls():
    names = declared_functions()
    for must in ("pnp_create", "pnp_cdft_mu_ex", "pnp_batch_mu_ex", "pnp_workspace_bytes",
                 "pnp_weighted_densities", "pnp_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTED) == declared_functions()


@pytest.mark.parametrize("n,ok", [(8, 1), (16, 1), (24, 1), (48, 1), (64, 1), (256, 1), (50, 0), (512, 0), (0, 0)])
def test_supported_sizes(n, ok):
    assert binding.load_library().pnp_supported_size(n) == ok


def test_create_without_device_reports_device_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    lib = binding.load_library()
    ctx = ctypes.c_void_p()
    assert lib.pnp_create(0, ctypes.byref(ctx)) == -7
    assert not ctx.value


def test_null_arguments_are_rejected_without_device():
    lib = binding.load_library()
    assert lib.pnp_create(0, None) == -1
    assert lib.pnp_workspace_bytes(None, None, 1, None, None) == -1


def test_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the binding's records equal what a C
    compiler makes of include/pnp_cdft.h (gcc on the host)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    recs = {"pnp_grid": binding.Grid, "pnp_species": binding.SpeciesC, "pnp_params": binding.ParamsC,
            "pnp_request": binding.RequestC, "pnp_relax_spec": binding.RelaxSpecC}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pnp_cdft.h"', 'int main(void) {']
    for cname, py in recs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            cf = "lambda" if fname == "lambda_" else fname
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (ln.split() for ln in out if ln.strip())}
    for cname, py in recs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def _uniform(problem, n=8):
    import numpy as np
    return np.stack([np.full((n, n, n), s.rho_bulk) for s in problem.species])


@pytest.mark.parametrize("terms", [1, 2, 4, 3, 5, 6, 7, 8, 14])
def test_bulk_mu_ex_against_oracle(terms):
    """pnp_bulk_mu_ex (host arithmetic behind the ABI, no device) equals the
    oracle's evaluation of uniform bulk densities, with non-zero EC bulk
    constants."""
    import numpy as np
    import oracle
    import pnp_inputs as P
    for prob, _ in (P.config1(), P.channel_problem(16, 7), P.config3(n=16)):
        sp = [P.Species(s.d, s.q, s.rho_bulk, 0.25 * (i + 1)) for i, s in enumerate(prob.species)]
        pr = prob.with_(terms=terms, species=sp, n=8)
        ref = oracle.mu_ex(pr, _uniform(pr), "fft")["total"][:, 0, 0, 0]
        got = np.array(pkg.bulk_mu_ex(pr))
        assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, float(np.max(np.abs(ref)))), (terms, got, ref)


def test_bulk_mu_ex_percus_yevick():
    """One hard-sphere species: the Rosenfeld bulk value is the Percus-Yevick
    compressibility result, -ln(1-eta) + (14 eta - 13 eta^2 + 5 eta^3) / (2 (1-eta)^3)."""
    import math
    import pnp_inputs as P
    eta, d = 0.45, 0.3
    sp = [P.Species(d, 0.0, eta / (math.pi / 6.0 * d ** 3))]
    pr = P.Problem(n=8, h=0.05, species=sp, T=300.0, terms=P.TERM_HS)
    py = -math.log(1 - eta) + (14 * eta - 13 * eta ** 2 + 5 * eta ** 3) / (2 * (1 - eta) ** 3)
    assert abs(pkg.bulk_mu_ex(pr)[0] - py) < 1e-12


def test_bulk_mu_ex_packing_error():
    import math
    import pnp_inputs as P
    sp = [P.Species(0.3, 0.0, 1.2 / (math.pi / 6.0 * 0.3 ** 3))]
    pr = P.Problem(n=8, h=0.05, species=sp, T=300.0, terms=P.TERM_HS)
    with pytest.raises(pkg.PnpError) as e:
        pkg.bulk_mu_ex(pr)
    assert e.value.status == -4


def test_pool_calls_reject_null():
    lib = binding.load_library()
    assert lib.pnp_pool_create(None, None, 0, None) == -1
    assert lib.pnp_session_step(None, 0, None, None, None) == -1
    assert lib.pnp_session_close(None, 1) == -1
    assert lib.pnp_pool_usage(None, None, None, None) == -1


@pytest.mark.parametrize("eta", [0.0, 0.02, 0.049, 0.051, 0.3, 0.45])
def test_bulk_mu_ex_carnahan_starling(eta):
    """One hard-sphere species with the White Bear functional: the bulk value
    is the Carnahan-Starling result (8 eta - 9 eta^2 + 3 eta^3) / (1 - eta)^3,
    on both sides of the switch between the series and the closed form."""
    import math
    import pnp_inputs as P
    d = 0.3
    sp = [P.Species(d, 0.0, eta / (math.pi / 6.0 * d ** 3))]
    pr = P.Problem(n=8, h=0.05, species=sp, T=300.0, terms=P.TERM_HS_WB)
    cs = (8 * eta - 9 * eta ** 2 + 3 * eta ** 3) / (1 - eta) ** 3
    assert abs(pkg.bulk_mu_ex(pr)[0] - cs) < 1e-13 * max(1.0, cs)


def test_hs_bits_are_exclusive():
    import pnp_inputs as P
    prob, _ = P.config1()
    for terms in (P.TERM_HS | P.TERM_HS_WB, 16, 0):
        with pytest.raises(pkg.PnpError) as e:
            pkg.bulk_mu_ex(prob.with_(terms=terms))
        assert e.value.status == -1


def test_bulk_mu_ex_bmcsl_mixture():
    """White Bear bulk values of a three-species mixture (host arithmetic
    behind the ABI) against the BMCSL closed form."""
    import numpy as np
    import pnp_inputs as P
    from test_oracle_fmt import bmcsl_mu
    ds, rb = (0.15, 0.3, 0.4), (3.0, 2.0, 4.0)
    pr = P.Problem(n=8, h=0.05, species=[P.Species(ds[i], 0.0, rb[i]) for i in range(3)], T=300.0,
                   terms=P.TERM_HS_WB)
    got = np.array(pkg.bulk_mu_ex(pr))
    ref = bmcsl_mu(ds, rb)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
