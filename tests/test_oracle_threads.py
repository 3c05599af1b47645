"""The OpenMP build of the oracle (same source, pixels of one colour shared among
threads) gives bitwise the single-threaded results: pixels of one colour read only the
other colour's state and their own within a half-sweep, and their random numbers are
keyed by pixel."""
import numpy as np
import pytest

import oracle
import scenegen as sg


@pytest.fixture(scope="module")
def scene():
    return sg.make_scene(17, sg.tiny_config(72, 56, n_src=3, n_planes=3, n_textureless=1), device="cpu")


def test_thread_count_in_effect():
    assert oracle.threads_in_effect(1) == 1
    assert oracle.threads_in_effect(4) == 4


@pytest.mark.parametrize("fp64", [False, True])
def test_threaded_patchmatch_is_bitwise(scene, fp64):
    pb = oracle.Problem.from_scene(scene, 7, 1, top_k=2)
    one = oracle.patchmatch(pb, 2, fp64=fp64, threads=1)
    many = oracle.patchmatch(pb, 2, fp64=fp64, threads=4)
    for a, b in zip(one, many):
        assert np.array_equal(a, b)


def test_threaded_init_halfsweep_and_cost_are_bitwise(scene):
    pb = oracle.Problem.from_scene(scene, 9, 2, top_k=0)
    P1, C1 = oracle.init(pb, threads=1)
    P4, C4 = oracle.init(pb, threads=4)
    assert np.array_equal(P1, P4) and np.array_equal(C1, C4)
    m = pb.valid_mask()
    sub = np.flatnonzero(m.ravel())[::3].astype(np.int32)
    for subset in (None, sub):
        a = oracle.halfsweep(pb, P1, C1, 1, 0, subset=subset, threads=1)
        b = oracle.halfsweep(pb, P1, C1, 1, 0, subset=subset, threads=4)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        a = oracle.eval_cost(pb, P1, subset=subset, threads=1)
        b = oracle.eval_cost(pb, P1, subset=subset, threads=4)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
