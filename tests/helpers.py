"""Shared helpers for the GPU parity tests (the only place oracle and library meet)."""
import numpy as np

from paper_2409_16675_amd import synth


def rand_planes(g, lead, q, N):
    return synth.uniform_residues(g, lead, q, N)


def assert_equal_u64(got, expect, what=""):
    got = np.asarray(got, dtype=np.uint64)
    expect = np.asarray(expect, dtype=np.uint64)
    assert got.shape == expect.shape, (what, got.shape, expect.shape)
    if not np.array_equal(got, expect):
        bad = np.argwhere(got != expect)
        first = tuple(bad[0])
        raise AssertionError("%s: %d mismatches, first at %s: got %d expected %d" %
                             (what, len(bad), first, int(got[first]), int(expect[first])))
