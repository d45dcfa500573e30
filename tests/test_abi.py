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


def test_check_sync_where_no_quick_witness_exists():
    """The synchronizability check first looks for a short reset word and
    otherwise runs the pair test: slowly synchronizing automata (Černý,
    reset threshold (n-1)^2, past the witness search's budget) and automata
    whose pairs merge only partly must still get the exact answer."""
    for n in (10, 40, 100, 200):
        assert srw.check_sync(n, 2, I.cerny(n))
        # the Černý shift with a second permutation instead of the merging letter
        d = np.asarray(I.cerny(n)).copy().reshape(2, n)
        d[0] = np.roll(np.arange(n), 2)
        assert not srw.check_sync(n, 2, d.reshape(-1))
        assert O.is_synchronizing(n, 2, I.cerny(n)) and not O.is_synchronizing(n, 2, d.reshape(-1))
    # two letters that merge inside two halves only: pairs across stay apart
    n = 60
    a = np.array([q - q % 2 for q in range(n)], np.int32)          # merges 2i, 2i+1
    b = np.array([(q + 2) % (n // 2) + (n // 2) * (q >= n // 2) for q in range(n)], np.int32)
    d = np.concatenate([a, b])
    assert srw.check_sync(n, 2, d) == O.is_synchronizing(n, 2, d) is False


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
    with pytest.raises(srw.SrwError) as e:
        srw.solve_noalloc(8, 2, d)
    assert e.value.code == srw.EDEVICE


def test_noalloc_host_checks_come_first():
    """The no-alloc entry point answers bad input, non-synchronizing input
    and n = 1 on the host, like srw_solve, before any device work."""
    with pytest.raises(srw.SrwError) as e:
        srw.solve_noalloc(3, 1, [0, 1, 5])
    assert e.value.code == srw.EINVAL
    with pytest.raises(srw.SrwError) as e:
        srw.solve_noalloc(3, 2, [1, 2, 0, 0, 2, 1])
    assert e.value.code == srw.ENOTSYNC
    assert srw.solve_noalloc(1, 2, [0, 0]) == (0, [])


def test_beam_host_checks_come_first():
    """srw_beam_batch answers bad input, non-synchronizing input and n = 1
    on the host, per automaton; a search that needs the GPU gets
    SRW_EDEVICE here (no GPU)."""
    res = srw.beam_batch([(3, 1, [0, 1, 5], 4), (3, 2, [1, 2, 0, 0, 2, 1], 4), (1, 2, [0, 0], 4),
                          (4, 2, I.cerny(4), 0)])
    assert [x[0] for x in res] == [srw.EINVAL, srw.ENOTSYNC, srw.OK, srw.EINVAL]
    assert res[2] == (srw.OK, 0, [])
    if not gpu_present():
        with pytest.raises(srw.SrwError) as e:
            srw.beam_batch([(4, 2, I.cerny(4), 4)])
        assert e.value.code == srw.EDEVICE


def test_eppstein_host_checks_come_first():
    """srw_eppstein_batch and srw_bound_batch answer bad input and n = 1 on
    the host, per automaton (a non-synchronizing automaton is found by the
    search over pairs on the device); a run that needs the GPU gets
    SRW_EDEVICE here (no GPU)."""
    res = srw.eppstein_batch([(3, 1, [0, 1, 5]), (1, 2, [0, 0])])
    assert [x[0] for x in res] == [srw.EINVAL, srw.OK]
    assert res[1] == (srw.OK, 0, [])
    res = srw.bound_batch([(3, 1, [0, 1, 5]), (1, 2, [0, 0])])
    assert [x[0] for x in res] == [srw.EINVAL, srw.OK]
    assert res[1] == (srw.OK, 0, 1, [])
    if not gpu_present():
        for f in (srw.eppstein_batch, srw.bound_batch):
            for d in (I.cerny(4), [1, 2, 3, 0, 0, 2, 1, 3]):
                with pytest.raises(srw.SrwError) as e:
                    f([(4, 2, d)])
                assert e.value.code == srw.EDEVICE


def test_estimator_inputs_generator_is_deterministic():
    a = I.random_automaton(100, 3, 12345, 2)
    b = I.random_automaton(100, 3, 12345, 2)
    assert np.array_equal(a, b)
    assert a.min() >= 0 and a.max() < 100
    # splitmix64 reference values of the published generator (seed 0)
    x = I.splitmix64_stream(0, 0, 3)
    assert [int(v) for v in x] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_every_documented_option_is_accepted_and_checked():
    """Each key the header documents is accepted with its default value;
    out-of-range values are SRW_EINVAL (no device needed to set options)."""
    import re
    with open(os.path.join(ROOT, "include", "srw.h")) as f:
        head = f.read()
    block = head[head.index("Tuning and test options"):head.index("int srw_set_option")]
    keys = re.findall(r'^ \*   "(\w+)"', block, re.M)
    defaults = {"budget": 0, "max_slots": 4096, "profile": 0, "schedule": 0, "sched_seed": 0,
                "meet": 0, "meet_tiles": 0, "meet_rows": 512, "meet_groups": 16, "meet_order": 1,
                "meet_grid": 0, "ysort": 0, "small_cand": 2048, "deadline_ms": 0,
                "verbose": 0, "keep_levels": 0, "persist": 1, "bucket": 16384, "meet_xcd": 0,
                "meet_bgrid": 4096, "reduce": 0}
    assert set(keys) == set(defaults), set(keys) ^ set(defaults)
    for k in keys:
        srw.set_option(k, defaults[k])
    bad = {"profile": 3, "schedule": 4, "meet": 3, "meet_order": 2, "meet_groups": 0,
           "meet_tiles": 1000, "ysort": -1, "small_cand": -1, "meet_grid": -1, "budget": -5,
           "persist": 2, "bucket": -1, "meet_xcd": -1, "meet_bgrid": 0, "reduce": 3}
    for k, v in bad.items():
        with pytest.raises(srw.SrwError) as e:
            srw.set_option(k, v)
        assert e.value.code == srw.EINVAL, k
        srw.set_option(k, defaults[k])


def test_per_width_options_are_checked():
    """"<key>@<W>" sets a value for one set width; bad widths, keys and
    values are SRW_EINVAL; -1 removes it."""
    for key, v in (("meet_groups@8", 32), ("meet_rows@1", 256), ("small_cand@3", 0),
                   ("bucket@5", 0), ("schedule@4", 3)):
        srw.set_option(key, v)
        srw.set_option(key, -1)
    for key, v in (("meet_groups@0", 16), ("meet_groups@9", 16), ("meet_groups@", 16),
                   ("meet_groups@12", 16), ("persist@2", 1), ("meet_groups@2", 0),
                   ("schedule@2", 4), ("small_cand@1", -2), ("bucket@1", -3)):
        with pytest.raises(srw.SrwError) as e:
            srw.set_option(key, v)
        assert e.value.code == srw.EINVAL, key


def test_last_sides_needs_a_kept_solve():
    with pytest.raises(srw.SrwError) as e:
        srw.last_sides()
    assert e.value.code == srw.EINVAL


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of srw_stats, srw_config and srw_result have the C
    sizes and field offsets (gcc on include/srw.h)."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    structs = {"srw_stats": srw.Stats, "srw_config": srw.Config, "srw_result": srw.Result}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "srw.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append('return 0; }')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        cname, what, val = line.split()
        py = structs[cname]
        want = ctypes.sizeof(py) if what == "size" else getattr(py, what).offset
        assert int(val) == want, (cname, what, int(val), want)
