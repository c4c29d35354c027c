"""The C-ABI library loads and exports every symbol its header declares (no GPU work)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="lba.h", prefix="lba_"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    pat = r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(" + prefix + r"[a-z_0-9]+)\s*\("
    return sorted(set(re.findall(pat, src, flags=re.M)))


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
    assert L.lba_abi_version() == 4
    assert L.lba_status_string(-5).decode() == "unsupported problem size"


def test_default_options_match_the_documented_values():
    from paper_2511_02036_amd import lba
    o = lba.default_options()
    assert (o.iters_round1, o.iters_round2, o.max_trials, o.round2_robust) == (5, 10, 10, 1)
    assert (o.huber2_mono, o.huber2_stereo, o.chi2_mono, o.chi2_stereo) == (5.991, 7.815, 5.991, 7.815)
    assert o.tau == 1e-5 and o.precision == lba.PREC_FP64
    assert o.trial_log == 0 and o.use_graphs == 1 and o.schur_fp32_accum == 0 and o.pair_cache == 1


def test_struct_layouts_match_the_header():
    """The ctypes mirrors have the sizes of the C structs (x86-64 System V layout)."""
    import ctypes as C
    from paper_2511_02036_amd import lba
    assert C.sizeof(lba.Options) == 6 * 4 + 5 * 8 + 5 * 4 + 4   # tail padding to 8 bytes
    assert C.sizeof(lba.TrialRecord) == 6 * 4 + 4 * 8
    assert C.sizeof(lba.Result) == 5 * 8


def test_library_exports_every_local_mapping_symbol():
    from paper_2511_02036_amd import lmap
    L = lmap.library()
    names = _declared("lmap.h", "lmap_")
    for must in ("lmap_index_build", "lmap_correspondence", "lmap_fusion", "lmap_culling"):
        assert must in names
    for name in names:
        assert hasattr(L, name), f"{name} declared in lmap.h but not exported"
    assert set(names) == set(lmap.EXPORTS)
    assert L.lmap_abi_version() == 1
    assert L.lmap_status_string(-4).decode() == "workspace too small"


def test_local_mapping_defaults_and_layouts():
    import ctypes as C
    from paper_2511_02036_amd import lmap
    p = lmap.corr_params()
    assert (p.th_low, p.resolve, p.epi_chi2, p.epipole_min) == (50, 1, 3.84, 100.0)
    f = lmap.fuse_params()
    assert (f.th_low, f.radius_th, f.chi2_mono, f.chi2_stereo) == (50, 3.0, 5.991, 7.815)
    c = lmap.cull_params()
    assert (c.min_obs, c.slack, c.num, c.den) == (3, 0, 9, 10)
    assert C.sizeof(lmap.Store) == 6 * 4 + 10 * 8 + 5 * 8
    assert C.sizeof(lmap.CorrParams) == 8 + 2 * 8
    assert C.sizeof(lmap.FuseParams) == 8 + 3 * 8
    assert C.sizeof(lmap.Points) == 8 + 5 * 8


def test_local_mapping_size_queries_need_no_gpu():
    """Workspace and index sizes are host arithmetic over the store's sizes."""
    import ctypes as C
    from paper_2511_02036_amd import lmap
    L = lmap.library()
    sig = (C.c_double * 8)(*[1.44 ** o for o in range(8)])
    sc = (C.c_double * 8)(*[1.2 ** o for o in range(8)])
    S = lmap.Store(80, 96000, 1200, 8, 752, 480, 1, 1, 1, 1, 1, 1, 1, None, C.addressof(sig), C.addressof(sc),
                   458.0, 458.0, 367.0, 248.0, 50.38)
    n = C.c_size_t()
    assert L.lmap_index_size(C.byref(S), C.byref(n)) == 0
    cells = 47 * 30
    a256 = lambda x: (x + 255) // 256 * 256
    assert n.value == a256(96000 * 256) + a256(80 * (cells + 1) * 4) + a256(96000 * 4) + 256
    assert L.lmap_corr_workspace_size(C.byref(S), 640, C.byref(n)) == 0
    assert n.value == 256 + a256(640 * 96) + a256(640 * 4) + a256(96000 * 4) + a256(80 * 4) + a256(640 * 1200 * 4)
    S.max_kp = 0
    assert L.lmap_index_size(C.byref(S), C.byref(n)) == -5
    S.max_kp = 1200
    S.width = 752 * 8
    assert L.lmap_index_size(C.byref(S), C.byref(n)) == -5
