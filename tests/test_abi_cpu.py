"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point declared in include/kmp.h, and reports argument errors."""
import ctypes
import os
import re

import pytest

import paper_2105_02022_amd as kmp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "kmp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kmp_[a-z_0-9]+)\s*\(", text)))


def test_library_present():
    assert os.path.exists(kmp.LIB_PATH), "build libkmp.so first (__graft_entry__.build())"


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(kmp.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(kmp.SIGNATURES)


def test_strerror_and_version():
    assert kmp.kmp_version().count(".") == 2
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert kmp.kmp_strerror(code)
    assert "unknown" in kmp.kmp_strerror(42)


def test_argument_errors_before_any_device_work():
    lib = kmp.library()
    # k < 1, n < 0, negative / NaN eps: rejected before touching memory
    assert lib.kmp_partition(None, None, None, None, 10, 0, 0, 0.03, 1, None, None) == kmp.KMP_EINVAL
    assert lib.kmp_partition(None, None, None, None, -1, 0, 2, 0.03, 1, None, None) == kmp.KMP_EINVAL
    assert lib.kmp_partition(None, None, None, None, 10, 0, 2, -1.0, 1, None, None) == kmp.KMP_EINVAL
    assert lib.kmp_partition(None, None, None, None, 10, 0, 2, float("nan"), 1, None, None) == kmp.KMP_EINVAL
    assert lib.kmp_partition(None, None, None, None, 10, 0, 2, 0.03, 1, None, None) == kmp.KMP_EINVAL  # NULL xadj
    # empty graph: OK without device work
    assert lib.kmp_partition(None, None, None, None, 0, 0, 4, 0.03, 1, None, None) == kmp.KMP_OK


def test_noalloc_limits_before_any_device_work():
    """kmp_partition_noalloc rejects inputs beyond its stated limits, and profiling, before touching
    the device; the header's limits and the binding's agree."""
    import ctypes
    import re
    lib = kmp.library()
    h = open(os.path.join(ROOT, "include", "kmp.h")).read()
    lim = {k: int(v) for k, v in re.findall(r"#define (KMP_NOALLOC_MAX_[NM]) (\d+)", h)}
    assert lim == {"KMP_NOALLOC_MAX_N": kmp.NOALLOC_MAX_N, "KMP_NOALLOC_MAX_M": kmp.NOALLOC_MAX_M}
    sc = re.search(r"#define KMP_NOALLOC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", h)
    assert int(sc.group(1)) << int(sc.group(2)) == kmp.NOALLOC_SCRATCH_BYTES
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the checks come first
    big_n, big_m = kmp.NOALLOC_MAX_N + 1, kmp.NOALLOC_MAX_M + 1
    assert lib.kmp_partition_noalloc(fake, fake, None, None, big_n, 0, 2, 0.03, 1, fake, None, None,
                                     None) == kmp.KMP_ETOOLARGE
    assert lib.kmp_partition_noalloc(fake, fake, None, None, 10, big_m, 2, 0.03, 1, fake, None, None,
                                     None) == kmp.KMP_ETOOLARGE
    opt = kmp.KmpOptions()
    opt.profile = 1
    assert lib.kmp_partition_noalloc(fake, fake, None, None, 10, 20, 2, 0.03, 1, fake, None, ctypes.byref(opt),
                                     None) == kmp.KMP_EINVAL
    assert lib.kmp_partition_noalloc(None, None, None, None, 10, 0, 0, 0.03, 1, None, None, None,
                                     None) == kmp.KMP_EINVAL
    assert lib.kmp_partition_noalloc(None, None, None, None, 0, 0, 4, 0.03, 1, None, None, None, None) == kmp.KMP_OK
    assert "limits" in kmp.kmp_strerror(kmp.KMP_ETOOLARGE)


def test_batch_argument_errors_before_any_device_work():
    lib = kmp.library()
    assert lib.kmp_partition_batch(None, -1, None, None, None, None) == kmp.KMP_EINVAL
    assert lib.kmp_partition_batch(None, 3, None, None, None, None) == kmp.KMP_EINVAL
    assert lib.kmp_partition_batch(None, 0, None, None, None, None) == kmp.KMP_OK


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the public structs have the sizes and offsets gcc gives the header's."""
    import subprocess
    fields = {"kmp_graph_desc": (kmp.KmpGraphDesc, ["n", "m", "seed", "out_part"]),
              "kmp_job_result": (kmp.KmpJobResult, ["cut", "lk", "level_n"]),
              "kmp_options": (kmp.KmpOptions, ["profile_classes", "force_exact", "small_level_n", "plain_loads",
                                               "fm_passes", "ip_pool", "pq_balance", "async_lp", "ip_multilevel"]),
              "kmp_stats": (kmp.KmpStats, ["lp_exact_subrounds", "level_n", "level_m", "ms_total", "prof_bytes"]),
              "kmp_server_stats": (kmp.KmpServerStats, ["hbm_in_use", "running_batches"]),
              "kmp_tuning": (kmp.KmpTuning, ["tier3_deg", "hub_lds_slots", "reserved"]),
              "kmp_autotune_report": (kmp.KmpAutotuneReport, ["ms_start", "ms_best"])}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "kmp.h"', "int main(void) {"]
    for st, (_, fs) in fields.items():
        lines.append(f'printf("%zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("%zu\\n", offsetof({st}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    exp = []
    for st, (cls, fs) in fields.items():
        exp.append(ctypes.sizeof(cls))
        exp += [getattr(cls, f).offset for f in fs]
    assert got == exp


def test_server_argument_errors_before_any_device_work():
    lib = kmp.library()
    assert not lib.kmp_server_create(1 << 30, 0)
    assert not lib.kmp_server_create(1 << 30, 17)
    assert not lib.kmp_server_create(0, 2)
    jid = ctypes.c_uint64(0)
    assert lib.kmp_server_submit(None, None, ctypes.byref(jid)) == kmp.KMP_EINVAL
    assert lib.kmp_server_poll(None, 1, None, None) == kmp.KMP_EINVAL
    assert lib.kmp_server_wait(None, 1, None, None) == kmp.KMP_EINVAL
    assert lib.kmp_server_stats_get(None, None) == kmp.KMP_EINVAL
    lib.kmp_server_destroy(None)


def test_tuning_validation_without_device_work():
    """kmp_set_tuning keeps the setting on a bad value; NULL restores the defaults."""
    lib = kmp.library()
    assert kmp.kmp_set_tuning(None) == kmp.KMP_OK
    dflt = kmp.kmp_get_tuning()
    assert dflt == {"small_level_n": 8192, "tier0_deg": 16, "tier1_deg": 64, "tier2_deg": 512, "tier3_deg": 4096,
                    "hub_lds_slots": 4096}
    bad = [dict(dflt, tier0_deg=17), dict(dflt, tier0_deg=0), dict(dflt, tier1_deg=8, tier0_deg=16),
           dict(dflt, tier2_deg=513), dict(dflt, tier3_deg=256), dict(dflt, small_level_n=-2),
           dict(dflt, small_level_n=(1 << 30) + 1), dict(dflt, hub_lds_slots=32), dict(dflt, hub_lds_slots=16384),
           dict(dflt, hub_lds_slots=1000)]
    for b in bad:
        assert kmp.kmp_set_tuning(b) == kmp.KMP_EINVAL, b
        assert kmp.kmp_get_tuning() == dflt
    good = dict(small_level_n=-1, tier0_deg=8, tier1_deg=32, tier2_deg=256, tier3_deg=2048, hub_lds_slots=64)
    assert kmp.kmp_set_tuning(good) == kmp.KMP_OK
    assert kmp.kmp_get_tuning() == good
    # a missing or zero hub_lds_slots is its default
    assert kmp.kmp_set_tuning(dict(good, hub_lds_slots=0)) == kmp.KMP_OK
    assert kmp.kmp_get_tuning() == dict(good, hub_lds_slots=4096)
    assert kmp.kmp_set_tuning(None) == kmp.KMP_OK
    assert kmp.kmp_get_tuning() == dflt
    assert lib.kmp_get_tuning(None) == kmp.KMP_EINVAL


def test_autotune_argument_errors_before_any_device_work():
    lib = kmp.library()
    assert lib.kmp_autotune(None, 3, None, None, None) == kmp.KMP_EINVAL
    d = kmp.KmpGraphDesc()
    d.n, d.k, d.m, d.epsilon = 10, 2, 0, 0.03
    assert lib.kmp_autotune(ctypes.byref(d), 0, None, None, None) == kmp.KMP_EINVAL   # reps
    assert lib.kmp_autotune(ctypes.byref(d), 51, None, None, None) == kmp.KMP_EINVAL  # reps
    assert lib.kmp_autotune(ctypes.byref(d), 3, None, None, None) == kmp.KMP_EINVAL   # NULL arrays
