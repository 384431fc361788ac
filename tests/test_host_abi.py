"""CPU-only checks of the C-ABI library: it loads, exports every entry point
the header declares, and its host-side spline layer (knot validation, Gauss
rule, 1D value/derivative tables) agrees with the oracle's independent
Cox-de Boor / numpy tables.  No GPU compute is issued here."""
import os
import re

import numpy as np
import pytest

import oracle
import paper_1809_05471_amd as sf
from paper_1809_05471_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "sfiga.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sf_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_header_symbol():
    L = sf.lib()
    declared = _header_functions()
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(sf.EXPORTED) == declared


def test_build_target():
    assert sf.sf_build_target() == "gfx950"


@pytest.mark.parametrize("p", range(2, 10))
@pytest.mark.parametrize("uniform", [True, False])
def test_host_tables_match_oracle(p, uniform):
    if uniform:
        kn = inputs.open_uniform_knots(7, p)
    else:
        inner = np.array([0.05, 0.2, 0.33, 0.5, 0.61, 0.9])
        kn = np.concatenate([np.zeros(p), inner, np.ones(p)])
    H = sf.sf_host_tables_1d(kn, p)
    O = oracle.tables_1d(kn, p)
    assert H["nel"] == O["nel"]
    assert np.all(O["first"] == np.arange(O["nel"]))
    assert np.abs(H["x"] - O["x"]).max() < 1e-15
    assert np.abs(H["w"] - O["w"]).max() < 1e-15
    assert np.abs(H["B"] - O["phi"]).max() < 1e-14
    scale = np.abs(O["dphi"]).max()
    assert np.abs(H["D"] - O["dphi"]).max() < 1e-13 * scale


def test_host_tables_error_paths():
    good = inputs.open_uniform_knots(4, 3)
    with pytest.raises(sf.SfError) as e:
        sf.sf_host_tables_1d(good[1:], 3)                     # not open at the left
    assert e.value.status == sf.SF_EKNOT
    bad = good.copy()
    bad[4], bad[5] = bad[5], bad[4]                          # decreasing
    with pytest.raises(sf.SfError) as e:
        sf.sf_host_tables_1d(bad, 3)
    assert e.value.status == sf.SF_EKNOT
    dbl = np.array([0, 0, 0, 0.5, 0.5, 1, 1, 1.0])           # double interior knot
    with pytest.raises(sf.SfError) as e:
        sf.sf_host_tables_1d(dbl, 3)
    assert e.value.status == sf.SF_EUNSUPPORTED
    with pytest.raises(sf.SfError) as e:
        sf.sf_host_tables_1d(good, 10)                       # order outside 2..9
    assert e.value.status == sf.SF_EUNSUPPORTED
    with pytest.raises(sf.SfError) as e:
        sf.sf_host_tables_1d(np.array([0, 0, 1, 1.0]), 3)     # too short
    assert e.value.status == sf.SF_EKNOT


def test_context_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(sf.SfError) as e:
        sf.sf_ctx_create(0, None)
    assert e.value.status in (sf.SF_EDEVICE, sf.SF_EINVAL)


def test_product_package_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1809_05471_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "orc.c" not in src and "liborc" not in src, f
