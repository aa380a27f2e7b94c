"""CPU checks of the C ABI: the library loads, exports every function the
public headers declare, and validates parameters on the host (no kernel
launches here)."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"\b(mlb_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_1105_3634_amd import _lib
    lib = _lib.load()
    declared = _declared()
    assert len(declared) >= 15
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly what the headers declare
    assert set(_lib.exported_symbols()) <= set(declared)


def test_workspace_size_and_validation():
    import paper_1105_3634_amd as mlb
    m, _, _ = W.config_bulk_diffusion()
    p = mlb.make_params(m, precision=32)
    nb = mlb.workspace_bytes(p)
    N, M = m.N, m.M
    assert nb > 4 * (2 * M * 19 * N)          # at least both population buffers
    p64 = mlb.make_params(m, precision=64)
    assert mlb.workspace_bytes(p64) > nb
    bad = [
        W.Mixture(3, 6, 6, sigma=(2.0, 3.0)),             # stencil reaches the box edge
        W.Mixture(8, 8, 8, sigma=(2.0, 3.0), tau=0.4),    # tau <= 1/2
        W.Mixture(8, 8, 8, sigma=(2.0, -1.0)),            # negative diameter
        W.Mixture(8, 8, 8, sigma=(2.0,), kT=0.5),         # kT must be 1/3
    ]
    for b in bad:
        with pytest.raises(mlb.MlbError) as e:
            mlb.workspace_bytes(mlb.make_params(b))
        assert e.value.status == -1
    asym = W.Mixture(16, 16, 16, sigma=(2.0, 3.0), eps=np.array([[0.1, 0.2], [0.1, 0.1]]))
    with pytest.raises(mlb.MlbError):
        mlb.workspace_bytes(mlb.make_params(asym))


def test_params_layout_matches_header():
    """Field order/size of mlb_params as parsed from the header."""
    from paper_1105_3634_amd import _lib
    src = open(os.path.join(ROOT, "include", "mlb.h")).read()
    body = re.search(r"typedef struct \{(.*?)\} mlb_params;", src, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(","):
            nm = re.findall(r"([A-Za-z_0-9]+)\s*(\[.*\])?\s*$", part.strip())
            names.append(nm[0][0])
    assert names == [f[0] for f in _lib.Params._fields_]
    assert ctypes.sizeof(_lib.Params) == 4 * 8 + 8 * (2 + 4 + 4 + 16 + 1 + 12 + 2)
