"""A context bound to the caller's HIP stream (nb_config.stream, here a
torch stream) gives the results of a context on the library's own stream,
bit for bit: construction steps, whose moment pass runs on the library's
second stream forked from and joined back into the caller's stream, reuse
steps, a tree built on its own, and a second construction."""
import numpy as np
import pytest
import torch

import workloads
import paper_1907_02290_amd as nb

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _ctx(d, order, stream=None):
    ctx = nb.Context(theta=0.5, eps=1 / 64, n_leaf=8, n_grp=64, order=order,
                     stream=stream)
    ctx.set_particles(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"],
                      d["m"])
    return ctx


def _same(a, b, what):
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v, err_msg=what)


@pytest.mark.parametrize("order", [1, 2])
def test_caller_stream_gives_the_same_results(order):
    # 2^19 Plummer particles, groups of at most 64: more than 8192 groups,
    # so the lists come from the split walk and the moment pass runs beside it
    say("case caller stream order=%d" % order)
    d = workloads.plummer(1 << 19, workloads.seed_for(3, 21))
    s = torch.cuda.Stream()
    own = _ctx(d, order)
    mine = _ctx(d, order, stream=s.cuda_stream)
    try:
        for ctx in (own, mine):
            ctx.build_tree()
        _same(own.get_moments(), mine.get_moments(), "moments, tree alone")
        assert own.get_info()["n_groups"] >= 8192
        dt = 1 / 512
        for step in range(8):
            mode = nb.NB_MAKE_LIST_FOR_REUSE if step % 4 == 0 else \
                nb.NB_REUSE_LIST
            for ctx in (own, mine):
                if step == 0:
                    ctx.compute_forces(mode)
                else:
                    ctx.step(mode, dt, dt)
            _same(own.get_forces(), mine.get_forces(), "forces, step %d" % step)
        _same(own.get_moments(), mine.get_moments(), "moments, last step")
    finally:
        own.close()
        mine.close()
        s.synchronize()
