"""The C-ABI library loads without a GPU and exports every entry point that
``include/nbody.h`` declares; argument checks that need no device work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(nb_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_step():
    names = _declared()
    for n in ("nb_create", "nb_destroy", "nb_set_particles", "nb_build_tree",
              "nb_make_lists", "nb_compute_forces", "nb_kick_drift",
              "nb_get_forces", "nb_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1907_02290_amd as nb
    lib = nb.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_version_string():
    import paper_1907_02290_amd as nb
    assert "gfx950" in nb.version()


@pytest.mark.parametrize("bad", [dict(theta=-0.1), dict(eps=0.0),
                                 dict(n_leaf=0), dict(n_leaf=65),
                                 dict(n_grp=0), dict(order=3),
                                 dict(theta=float("nan"))])
def test_create_rejects_bad_config_before_touching_the_device(bad):
    import paper_1907_02290_amd as nb
    kw = dict(theta=0.5, eps=0.01, n_leaf=8, n_grp=64, order=1)
    kw.update(bad)
    with pytest.raises(nb.NbError) as e:
        nb.Context(**kw)
    assert e.value.code == nb.NB_ERR_INPUT


def test_null_context_is_rejected():
    import paper_1907_02290_amd as nb
    lib = nb.load()
    assert lib.nb_build_tree(None) == nb.NB_ERR_INPUT
    assert lib.nb_compute_forces(None, 0) == nb.NB_ERR_INPUT
    assert lib.nb_kick_drift(None, 0.1, 0.1) == nb.NB_ERR_INPUT
    lib.nb_destroy(None)  # no-op


def test_binding_constants_match_the_header():
    import paper_1907_02290_amd as nb
    src = open(HEADER).read()
    for name, val in (("NB_MLP_NIN", nb.MLP_NIN),
                      ("NB_MLP_NPARAM", nb.MLP_NPARAM),
                      ("NB_MLP_STATIC_MAX_ROWS", nb.MLP_STATIC_MAX_ROWS)):
        m = re.search(r"\b%s\s*=\s*(\d+)" % name, src)
        assert m and int(m.group(1)) == val, name
