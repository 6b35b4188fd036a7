"""The D3Q19 transform header is what its generator emits today, and the
generator's symbolic checks (each emitted function equals its definition:
r = M d, k = N(u) r, r = N(u)^-1 k for zero first central moments,
d = M^-1 r) pass."""
import contextlib
import importlib.util
import io
import os

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2602_16486_amd", "csrc")


def test_header_is_current():
    pytest.importorskip("sympy")
    spec = importlib.util.spec_from_file_location("gen_d3q19", os.path.join(CSRC, "gen_d3q19.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    out = io.StringIO()
    with contextlib.redirect_stdout(out):
        gen.main()
    with open(os.path.join(CSRC, "cmflb_d3q19.h")) as fh:
        committed = fh.read()
    assert out.getvalue().rstrip("\n") == committed.rstrip("\n")
