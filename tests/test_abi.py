"""The C-ABI library loads and exports every symbol its header declares (no GPU work)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lba.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(lba_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("lba_create", "lba_solve", "lba_destroy", "lba_solve_batch", "lba_workspace_size"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2511_02036_amd import lba
    L = lba.library()
    for name in _declared():
        assert hasattr(L, name), f"{name} declared in lba.h but not exported"
    assert set(_declared()) <= set(lba.EXPORTS)
    assert L.lba_abi_version() == 2
    assert L.lba_status_string(-5).decode() == "unsupported problem size"


def test_default_options_match_the_documented_values():
    from paper_2511_02036_amd import lba
    o = lba.default_options()
    assert (o.iters_round1, o.iters_round2, o.max_trials, o.round2_robust) == (5, 10, 10, 1)
    assert (o.huber2_mono, o.huber2_stereo, o.chi2_mono, o.chi2_stereo) == (5.991, 7.815, 5.991, 7.815)
    assert o.tau == 1e-5 and o.precision == lba.PREC_FP64
    assert o.trial_log == 0 and o.use_graphs == 1


def test_struct_layouts_match_the_header():
    """The ctypes mirrors have the sizes of the C structs (x86-64 System V layout)."""
    import ctypes as C
    from paper_2511_02036_amd import lba
    assert C.sizeof(lba.Options) == 6 * 4 + 5 * 8 + 3 * 4 + 4
    assert C.sizeof(lba.TrialRecord) == 6 * 4 + 4 * 8
    assert C.sizeof(lba.Result) == 5 * 8
