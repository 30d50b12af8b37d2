"""Host logic of the server that needs no GPU: batch formation and arrivals."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2403_10647_amd import serve  # noqa: E402


class _Inp:
    def __init__(self, ncells, ntris=0):
        self.ncells = ncells
        self.ntris = ntris


def _req(i, npairs, ncells):
    r = serve.Request(i, 0.0, _Inp(ncells))
    r.npairs = npairs
    r.out_bytes = serve.output_bytes(npairs, ncells)
    return r


def test_bits_for():
    assert [serve.bits_for(n) for n in (0, 1, 2, 3, 4, 5, 1 << 20, (1 << 20) + 1)] == [0, 0, 1, 2, 2, 3, 20, 21]


def test_output_bytes():
    assert serve.output_bytes(0, 10) == 8 + 80
    assert serve.output_bytes(100, 10) == 800 + 80


def test_form_batch_limits():
    q = [_req(i, 100, 64) for i in range(10)]
    big = 1 << 40
    assert serve.form_batch(q, big, 512, 1 << 30) == 10
    assert serve.form_batch(q, big, 4, 1 << 30) == 4                  # grid cap
    assert serve.form_batch(q, big, 512, 350) == 3                    # pair cap
    assert serve.form_batch(q, 3 * q[0].out_bytes, 512, 1 << 30) == 3  # byte budget
    assert serve.form_batch(q, q[0].out_bytes - 1, 512, 1 << 30) == 0  # the head does not fit
    assert serve.form_batch([], big, 512, 1 << 30) == 0


def test_form_batch_head_may_exceed_pair_cap():
    q = [_req(0, 10_000, 8), _req(1, 10, 8)]
    assert serve.form_batch(q, 1 << 40, 512, 100) == 1


def test_form_batch_keeps_keys_within_32_bits():
    # the cells of a batch's grids are numbered in one 32-bit space
    q = [_req(i, 1, 1 << 27) for i in range(40)]
    assert serve.form_batch(q, 1 << 50, 512, 1 << 30) == 32
    q = [_req(i, 1, 1 << 30) for i in range(5)]
    assert serve.form_batch(q, 1 << 50, 512, 1 << 30) == 4
    q = [_req(i, 1, 1 << 10) for i in range(100)] + [_req(100, 1, 1 << 30)] * 4
    assert serve.form_batch(q, 1 << 50, 512, 1 << 30) == 103   # 100 * 2^10 + 3 * 2^30 < 2^32


def _arr(i, ntris, ncells=64):
    return serve.Request(i, 0.0, _Inp(ncells, ntris))


def test_form_count_batch_limits():
    # before the count only the triangles are known: pairs are predicted at a pairs-per-triangle rate
    a = [_arr(i, 1000) for i in range(10)]
    assert serve.form_count_batch(a, 512, 1 << 30, 4.0) == 10
    assert serve.form_count_batch(a, 3, 1 << 30, 4.0) == 3                # grid cap
    assert serve.form_count_batch(a, 512, 12_000, 4.0) == 3               # 3 x 4000 predicted pairs fit
    assert serve.form_count_batch(a, 512, 11_999, 4.0) == 2
    assert serve.form_count_batch(a, 512, 100, 4.0) == 1                  # the head always goes
    assert serve.form_count_batch([], 512, 1 << 30, 4.0) == 0
    q = [_arr(i, 1, 1 << 30) for i in range(5)]
    assert serve.form_count_batch(q, 512, 1 << 30, 4.0) == 4              # 32-bit cell space


def test_poisson_arrivals():
    t = serve.poisson_arrivals(2000.0, 5.0, seed=0)
    assert np.all(np.diff(t) > 0) and t[0] >= 0 and t[-1] < 5.0
    assert abs(len(t) - 10_000) < 5 * np.sqrt(10_000)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 2000) < 0.05 / 2000
    assert np.array_equal(t, serve.poisson_arrivals(2000.0, 5.0, seed=0))
    assert not np.array_equal(t[:100], serve.poisson_arrivals(2000.0, 5.0, seed=1)[:100])
