"""Host-side checks of libsrw that need no GPU: the library loads, it
exports every entry point include/srw.h declares, its host-only calls
(synchronizability test, word verification) agree with the oracle, argument
errors come back as status codes, and without a GPU a solve fails loudly."""

import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_05495_amd import inputs as I
from paper_2207_05495_amd import srw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "srw.h")


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w ]+?\**)\s*\**(srw_\w+)\s*\(", txt, re.M)))


def gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def test_header_lists_the_binding_exports():
    assert declared_symbols() == sorted(srw.EXPORTS)


def test_one_hip_runtime_in_process():
    """The binding loads libsrw after torch, so the process maps a single
    HIP runtime (two HSA runtimes in one process leave the second one without
    a device)."""
    srw.load()
    maps = {line.split()[-1] for line in open("/proc/self/maps") if "libamdhip64" in line}
    assert len(maps) == 1, maps


def test_library_exports_every_declared_symbol():
    lib = srw.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_check_sync_matches_oracle():
    seen = [0, 0]
    for i in range(300):
        n, k = 2 + i % 12, 1 + i % 3
        d = I.random_automaton(n, k, I.member_seed(4321, i))
        s = srw.check_sync(n, k, d)
        assert s == O.is_synchronizing(n, k, d)
        seen[s] += 1
    for n in (64, 200, 512):
        d = I.random_automaton(n, 2, I.member_seed(99, n))
        assert srw.check_sync(n, 2, d) == O.is_synchronizing(n, 2, d)
    assert srw.check_sync(40, 2, I.cerny(40))
    assert seen[0] > 10 and seen[1] > 100


def test_verify_matches_oracle():
    for n in (3, 16, 64, 65):
        d, _ = I.first_synchronizing(n, 2, I.member_seed(1, n), O.is_synchronizing)
        r, w, _ = O.bidir(n, 2, d)
        assert srw.verify(n, 2, d, w)
        if r > 0:
            assert not srw.verify(n, 2, d, w[:-1])
    assert srw.verify(1, 1, [0], [])


def test_bad_arguments_are_status_codes():
    with pytest.raises(srw.SrwError) as e:
        srw.check_sync(3, 1, [0, 1, 5])
    assert e.value.code == srw.EINVAL
    with pytest.raises(srw.SrwError) as e:
        srw.check_sync(600, 1, np.zeros(600, np.int32))
    assert e.value.code == srw.EUNSUPPORTED
    with pytest.raises(srw.SrwError) as e:
        srw.solve(0, 1, [0])
    assert e.value.code == srw.EINVAL
    with pytest.raises(srw.SrwError) as e:
        srw.set_option("no_such_option", 1)
    assert e.value.code == srw.EINVAL
    with pytest.raises(srw.SrwError) as e:
        srw.solve(3, 2, [1, 2, 0, 0, 2, 1])      # two permutations
    assert e.value.code == srw.ENOTSYNC


def test_trivial_cases_need_no_device():
    # n = 1 is answered before any device work: r = 0, empty word
    assert srw.solve(1, 3, [0, 0, 0]) == (0, [])


@pytest.mark.skipif(gpu_present(), reason="checks the no-GPU failure path")
def test_solve_without_gpu_fails_loudly():
    d = I.cerny(8)
    with pytest.raises(srw.SrwError) as e:
        srw.solve(8, 2, d)
    assert e.value.code == srw.EDEVICE
    with pytest.raises(srw.SrwError) as e:
        srw.Server()
    assert e.value.code == srw.EDEVICE


def test_estimator_inputs_generator_is_deterministic():
    a = I.random_automaton(100, 3, 12345, 2)
    b = I.random_automaton(100, 3, 12345, 2)
    assert np.array_equal(a, b)
    assert a.min() >= 0 and a.max() < 100
    # splitmix64 reference values of the published generator (seed 0)
    x = I.splitmix64_stream(0, 0, 3)
    assert [int(v) for v in x] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
