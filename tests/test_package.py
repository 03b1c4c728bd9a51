"""The package exports every name the binding defines for callers."""
import paper_1907_02290_amd as pkg
from paper_1907_02290_amd import nbody


def test_exports_cover_the_binding_constants():
    for name in dir(nbody):
        if name.startswith(("NB_", "MLP_")):
            assert getattr(pkg, name) == getattr(nbody, name), name
    assert pkg.MLP_NPARAM == 12 * 64 + 64 + 64 * 64 + 64 + 64 + 1
