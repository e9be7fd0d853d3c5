"""The C ABI library builds for gfx950, loads, exports every function that
include/h4d.h declares, and its struct layouts agree with the binding.
No compute call is made here (no GPU in this environment)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2307_11447_amd import h4d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "h4d.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(h4d_\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = h4d.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def test_library_is_built_for_gfx950():
    # the embedded HIP fat binary names its offload target
    blob = open(h4d.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_struct_layouts_match_header():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "h4d.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(h4d_params), sizeof(h4d_trial),
         sizeof(h4d_observables), offsetof(h4d_params, seed), offsetof(h4d_trial, dH), offsetof(h4d_observables, U),
         sizeof(h4d_timing), offsetof(h4d_trial, trial), sizeof(h4d_checkpoint), offsetof(h4d_checkpoint, trial),
         offsetof(h4d_checkpoint, n_trials));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, c], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == [C.sizeof(h4d.Params), C.sizeof(h4d.Trial), C.sizeof(h4d.Observables),
                    h4d.Params.seed.offset, h4d.Trial.dH.offset, h4d.Observables.U.offset,
                    C.sizeof(h4d.Timing), h4d.Trial.trial.offset, C.sizeof(h4d.Checkpoint),
                    h4d.Checkpoint.trial.offset, h4d.Checkpoint.n_trials.offset]


def test_invalid_parameters_are_rejected_before_any_device_work():
    from paper_2307_11447_amd import workloads as W
    w = W.small_lj(64, 0.3, 1)
    bad = dict(w.params, n_types=0)
    with pytest.raises(h4d.H4DError) as e:
        h4d.System(bad, w.x, w.type, w.mol, w.tag, w.nsalt, stream=C.c_void_p())
    assert e.value.code == h4d.H4D_EINVAL
    small_box = dict(w.params, box=[5.0, 5.0, 5.0])
    with pytest.raises(h4d.H4DError) as e:
        h4d.System(small_box, w.x % 5.0, w.type, w.mol, w.tag, w.nsalt, stream=C.c_void_p())
    assert e.value.code == h4d.H4D_EINVAL


def test_momentum_options_are_validated_before_any_device_work():
    from paper_2307_11447_amd import workloads as W
    w = W.small_lj(64, 0.3, 1)
    for bad in (dict(w.params, momenta=2), dict(w.params, md_refresh=1.5), dict(w.params, md_refresh=-0.1)):
        with pytest.raises(h4d.H4DError) as e:
            h4d.System(bad, w.x, w.type, w.mol, w.tag, w.nsalt, stream=C.c_void_p())
        assert e.value.code == h4d.H4D_EINVAL
    with pytest.raises(h4d.H4DError) as e:   # carried momenta need an ion system
        h4d.System(dict(w.params, momenta=1, water=1), w.x, w.type, w.mol, w.tag, w.nsalt, stream=C.c_void_p())
    assert e.value.code == h4d.H4D_EINVAL


def test_bench_refuses_more_than_one_gpu():
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_checkpoint_record_of_the_wrong_size_is_refused():
    good = np.zeros(C.sizeof(h4d.Checkpoint), np.uint8)
    assert isinstance(h4d._checkpoint_record({"checkpoint": good}), h4d.Checkpoint)
    with pytest.raises(ValueError):
        h4d._checkpoint_record({"checkpoint": good[:-8]})


def test_setters_refuse_a_null_handle_and_bad_modes():
    lib = h4d.lib()
    assert lib.h4d_set_list_loads(None, 0) == h4d.H4D_EINVAL
    assert lib.h4d_set_timing(None, 1) == h4d.H4D_EINVAL
    timing = h4d.Timing()
    assert lib.h4d_get_timing(None, C.byref(timing)) == h4d.H4D_EINVAL
