"""The seeded input generators (CPU): the batched chain generator gives the
per-instance draws bit for bit and runs inside the calling process."""
import multiprocessing
import threading

import numpy as np

from paper_2311_07602_amd import inputs


def test_chain_instances_equal_per_instance_draws():
    count, b, r = 200, 96, 12
    h = inputs.chain_instances(2, count, b, r, chunk=16, threads=4)
    assert h.shape == (count, 4, r, b)
    for i in (0, 1, 15, 16, 77, 199):
        ci = inputs.chain_instance(2, i, b, r)
        for t, x in enumerate((ci.U1, ci.V1, ci.U2, ci.V2)):
            assert np.array_equal(h[i, t], x.T), (i, t)


def test_chain_instances_independent_of_chunking():
    a = inputs.chain_instances(2, 37, 64, 8, chunk=5, threads=3)
    b = inputs.chain_instances(2, 37, 64, 8, chunk=64, threads=1)
    assert np.array_equal(a, b)


def test_chain_instances_start_no_process():
    before = set(multiprocessing.active_children())
    threads_before = threading.active_count()
    inputs.chain_instances(2, 300, 64, 8)
    assert set(multiprocessing.active_children()) == before
    assert threading.active_count() == threads_before
