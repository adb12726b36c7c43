"""Front end of run-time compiled systems, CPU only: the generated source
compiles with hipRTC (no device needed), the volume flux it describes has the
oracle's flux matrices, and malformed expressions are refused."""
import numpy as np
import pytest

from oracle import linear as Li

dg = pytest.importorskip("paper_1211_0582_amd.dg", reason="libdg.so not built")
from paper_1211_0582_amd import systems as S  # noqa: E402


@pytest.mark.parametrize("name,N,precision", [("acoustics", 1, "fp64"), ("acoustics", 9, "fp32"),
                                               ("maxwell", 4, "fp64"), ("advection", 2, "fp32")])
def test_generated_source_compiles(name, N, precision):
    spec = {"acoustics": S.acoustics(), "maxwell": S.maxwell(), "advection": S.advection((1.0, -0.5, 0.25))}[name]
    S.dg.dg_system_compile(spec.source(), spec.M, N, precision, "gfx950")


def test_flux_matrices_match_the_oracle():
    assert np.array_equal(S.flux_matrices(S.acoustics()), Li.acoustics_system().A)
    assert np.array_equal(S.flux_matrices(S.maxwell()), Li.maxwell_system().A)


def test_bad_source_is_refused_with_the_compiler_log():
    with pytest.raises(dg.DgError) as e:
        dg.dg_system_compile("struct System { static constexpr int M = 2; };", 2, 3, "fp64", "gfx950")
    assert e.value.status == dg.DG_EINVAL and "does not compile" in str(e.value)
    spec = S.acoustics()
    with pytest.raises(dg.DgError) as e:              # System::M differs from nfields
        dg.dg_system_compile(spec.source(), 3, 3, "fp64", "gfx950")
    assert e.value.status == dg.DG_EINVAL
    with pytest.raises(dg.DgError) as e:
        dg.dg_system_compile(spec.source(), 4, 3, "bf16x3", "gfx950")
    assert e.value.status == dg.DG_EUNSUPPORTED


@pytest.mark.parametrize("expr", ["p_m + q_m", "__import__('os')", "p_m ** 2", "lambda: 1", "p_m if nx else 0"])
def test_expressions_outside_the_grammar_are_refused(expr):
    spec = S.SystemSpec("bad", ("p",), {"x": {"p": "p"}}, {"p": expr}, {})
    with pytest.raises(S.ExpressionError):
        spec.source()
