"""Host-side checks of the C ABI (include/z4c.h) that need no GPU: the library
loads, exports every declared function, reports its defaults and tile set,
and rejects invalid arguments with the documented status before it would
enqueue anything.  Every call below has at least one invalid argument, so no
HIP call is reached."""
import ctypes
import json
import os

import pytest

from paper_2607_08743_amd import z4c

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "params.json")))
FAKE = ctypes.c_void_p(0x10000)       # never dereferenced: validation fails first
FAKE2 = ctypes.c_void_p(0x7F0000000)


@pytest.fixture(scope="module")
def L():
    return z4c.lib()


def test_every_declared_function_is_exported(L):
    names = z4c.header_functions()
    for required in ("rhs_z4c", "rk4_substep", "apply_ghosts", "z4c_plan_create", "z4c_plan_step",
                     "z4c_plan_autotune", "z4c_plan_destroy", "z4c_default_params", "z4c_last_error"):
        assert required in names
    for n in names:
        assert hasattr(L, n), n


def test_default_params_match_paper(L):
    p = z4c.default_params()
    for k in ("kappa1", "kappa2", "eta", "ko_sigma", "shift_coeff"):
        assert getattr(p, k) == GOLDEN[k]["value"]
    assert p.kappa3 == 0.0 and p.lapse_uses_K == 0 and p.precision == z4c.FP64


def test_tiles_enumerate(L):
    for prec in (z4c.FP64, z4c.MIXED):
        ts = z4c.tiles(prec)
        assert len(ts) >= 1
        for t in ts:
            assert t.bx * t.by * t.bz <= 1024 and t.waves in (1, 2)
    bad = z4c.Tile(3, 3, 3, 1, 0)
    assert L.z4c_select_tile(z4c.FP64, ctypes.byref(bad)) == z4c.EUNSUPPORTED
    assert L.z4c_select_tile(7, None) == z4c.EINVAL
    assert L.z4c_tile_get(z4c.FP64, 999, ctypes.byref(bad)) == z4c.EINVAL


def test_tile_resources_validation(L):
    """z4c_tile_resources refuses bad arguments before any HIP call."""
    w, s, x = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    good = z4c.Tile(8, 8, 8, 2, 1)
    assert L.z4c_tile_resources(7, ctypes.byref(good), ctypes.byref(w), ctypes.byref(s), ctypes.byref(x)) == z4c.EINVAL
    assert L.z4c_tile_resources(z4c.FP64, None, ctypes.byref(w), ctypes.byref(s), ctypes.byref(x)) == z4c.EINVAL
    assert L.z4c_tile_resources(z4c.FP64, ctypes.byref(good), None, ctypes.byref(s), ctypes.byref(x)) == z4c.EINVAL
    bad = z4c.Tile(3, 3, 3, 1, 0)
    assert L.z4c_tile_resources(z4c.FP64, ctypes.byref(bad), ctypes.byref(w), ctypes.byref(s),
                                ctypes.byref(x)) == z4c.EUNSUPPORTED


def _rhs(L, p, u=FAKE, r=FAKE2, sf=100000, n=(8, 8, 8), ng=3, h=(0.1, 0.1, 0.1), bc=0):
    return L.rhs_z4c(u, r, sf, n[0], n[1], n[2], ng, h[0], h[1], h[2], 0.0, 0.0, 0.0, bc, ctypes.byref(p), None)


@pytest.mark.parametrize("case", ["ng2", "nx0", "bc", "sf", "dx", "nan_dx", "null_u", "alias", "precision",
                                  "wfloor", "huge"])
def test_rhs_validation(L, case):
    p = z4c.default_params()
    kw = {}
    if case == "ng2":
        kw = dict(ng=2)
    elif case == "nx0":
        kw = dict(n=(0, 8, 8))
    elif case == "bc":
        kw = dict(bc=5)
    elif case == "sf":
        kw = dict(sf=14 ** 3 - 1)
    elif case == "dx":
        kw = dict(h=(0.1, 0.0, 0.1))
    elif case == "nan_dx":
        kw = dict(h=(0.1, float("nan"), 0.1))
    elif case == "null_u":
        kw = dict(u=None)
    elif case == "alias":
        kw = dict(r=ctypes.c_void_p(0x10000 + 8 * 1000))
    elif case == "precision":
        p.precision = 9
    elif case == "wfloor":
        p.w_floor = 0.0
    elif case == "huge":
        kw = dict(n=(2000, 2000, 2000), sf=2 ** 40)
    assert _rhs(L, p, **kw) == z4c.EINVAL
    assert len(L.z4c_last_error()) > 0


@pytest.mark.parametrize("case", ["stage0", "stage5", "dt0", "dt_nan", "out_is_in", "acc_is_in", "out_is_un_stage2",
                                  "no_un_stage2", "null_acc"])
def test_rk4_substep_validation(L, case):
    p = z4c.default_params()
    stage, dt = 2, 0.05
    u_in, u_n, acc, out = FAKE, ctypes.c_void_p(0x20000000), ctypes.c_void_p(0x40000000), ctypes.c_void_p(0x60000000)
    if case == "stage0":
        stage = 0
    elif case == "stage5":
        stage = 5
    elif case == "dt0":
        dt = 0.0
    elif case == "dt_nan":
        dt = float("nan")
    elif case == "out_is_in":
        out = u_in
    elif case == "acc_is_in":
        acc = u_in
    elif case == "out_is_un_stage2":
        out = u_n
    elif case == "no_un_stage2":
        u_n = None
    elif case == "null_acc":
        acc = None
    rc = L.rk4_substep(stage, dt, u_in, u_n, acc, out, 14 ** 3, 8, 8, 8, 3, 0.1, 0.1, 0.1, 0.0, 0.0, 0.0, 0,
                       ctypes.byref(p), None)
    assert rc == z4c.EINVAL, z4c.lib().z4c_last_error()


def test_apply_ghosts_validation(L):
    sf = 14 ** 3
    assert L.apply_ghosts(None, None, sf, 8, 8, 8, 3, 0, None) == z4c.EINVAL
    assert L.apply_ghosts(FAKE, None, sf, 8, 8, 8, 3, 2, None) == z4c.EINVAL      # copy without shell
    assert L.apply_ghosts(FAKE, FAKE2, sf, 8, 8, 8, 3, 0, None) == z4c.EINVAL     # shell on periodic box
    assert L.apply_ghosts(FAKE, FAKE, sf, 8, 8, 8, 3, 2, None) == z4c.EINVAL      # shell overlaps u
    assert L.apply_ghosts(FAKE, None, sf, 8, 8, 8, 1, 0, None) == z4c.EINVAL      # ng < 3
    # a Sommerfeld box has nothing to fill: accepted without touching memory
    assert L.apply_ghosts(FAKE, None, sf, 8, 8, 8, 3, 1, None) == z4c.OK


def test_plan_validation(L):
    p = z4c.default_params()
    h = ctypes.c_void_p()
    b = z4c.Box()
    b.n[:] = [8, 8, 8]
    b.ng, b.bc, b.sf = 3, 0, 14 ** 3
    b.dx[:] = [0.1, 0.1, 0.1]
    b.dt = 0.05
    b.u_n, b.u_a, b.u_b, b.acc = 0x10000000, 0x20000000, 0x30000000, 0x40000000
    arr = (z4c.Box * 1)(b)
    assert L.z4c_plan_create(arr, 0, ctypes.byref(p), None, None, ctypes.byref(h)) == z4c.EINVAL
    assert L.z4c_plan_create(arr, 17, ctypes.byref(p), None, None, ctypes.byref(h)) == z4c.EINVAL
    arr[0].u_b = arr[0].u_a
    assert L.z4c_plan_create(arr, 1, ctypes.byref(p), None, None, ctypes.byref(h)) == z4c.EINVAL
    assert b"overlap" in L.z4c_last_error()
    arr[0].u_b = 0x30000000
    arr[0].bc = 2  # copy box without shell
    assert L.z4c_plan_create(arr, 1, ctypes.byref(p), None, None, ctypes.byref(h)) == z4c.EINVAL
    assert L.z4c_plan_step(None, 1, 1, None) == z4c.EINVAL
    assert L.z4c_plan_destroy(None) == z4c.EINVAL
    assert L.z4c_plan_tile(None, None, None) == z4c.EINVAL


def _tune_boxes(n=(8, 8, 8), count=1):
    arr = (z4c.Box * count)()
    for c in arr:
        c.n[:] = list(n)
        c.ng, c.bc, c.sf = 3, 0, (n[0] + 6) * (n[1] + 6) * (n[2] + 6)
        c.dx[:] = [0.1, 0.1, 0.1]
        c.dt = 0.05
    for k, c in enumerate(arr):
        c.u_n, c.u_a, c.u_b, c.acc = [0x10000000 * (4 * k + i + 1) for i in range(4)]
    return arr


def test_tune_cache_lookup_hit_miss_missing_corrupt(L, tmp_path):
    """The tuning cache (JSON lines keyed by architecture, precision, box
    count and bucket = floor(log2(active cells))): hit, key misses, a missing
    file (an empty cache), a corrupt file (Z4C_EINVAL) and a cached shape this
    build does not compile (a miss)."""
    from paper_2607_08743_amd import inputs as I
    path = tmp_path / "tune.jsonl"
    g256 = I.centered_grid(256, 0.125)
    t = z4c.tiles(z4c.FP64)[0]
    path.write_text(json.dumps({"arch": "gfx950", "precision": 0, "nbox": 1, "bucket": 24,
                                "tile": [t.bx, t.by, t.bz, t.waves, 1], "ms": 29.4}) + "\n\n"
                    + json.dumps({"arch": "gfx950", "precision": 1, "nbox": 1, "bucket": 24,
                                  "tile": [3, 3, 3, 1, 0], "ms": 1.0}) + "\n")
    hit = z4c.tune_lookup(str(path), "gfx950", [g256])
    assert hit is not None and hit.as_tuple() == (t.bx, t.by, t.bz, t.waves, 1)
    assert z4c.tune_lookup(str(path), "gfx942", [g256]) is None                    # other architecture
    assert z4c.tune_lookup(str(path), "gfx950", [I.centered_grid(128, 0.25)]) is None  # other bucket (21)
    assert z4c.tune_lookup(str(path), "gfx950", [g256, g256]) is None              # other box count
    assert z4c.tune_lookup(str(path), "gfx950", [g256], z4c.MIXED) is None         # shape not compiled
    # the bucket is floor(log2(cells)): 2^24 - 1 cells fall in bucket 23
    assert z4c.tune_lookup(str(path), "gfx950", [I.centered_grid((256, 256, 255), 0.125)]) is None
    assert z4c.tune_lookup(str(tmp_path / "missing.jsonl"), "gfx950", [g256]) is None
    for bad in ('{"arch": "gfx950", "precision": 0, "nbox": 1, "bucket": 24}',            # no tile
                '{"arch": "gfx950", "precision": 0, "nbox": 1, "bucket": 24, "tile": [8, 8]}',
                '{"arch": "gfx950", "precision": 0, "nbox": 1, "bucket": 24, "tile": [8,8,8,2,1], "x": 1}',
                'not json at all', '{"arch": "gfx950"'):
        path.write_text(bad + "\n")
        with pytest.raises(z4c.Z4cError) as ei:
            z4c.tune_lookup(str(path), "gfx950", [g256])
        assert ei.value.status == z4c.EINVAL and b"tune cache" in L.z4c_last_error()


def test_plan_create_with_tune_cache(L, tmp_path):
    """z4c_plan_create with a cache path: a missing file is an empty cache
    (default tile, no HIP call needed), a corrupt one fails with Z4C_EINVAL
    before anything else happens."""
    p = z4c.default_params()
    h = ctypes.c_void_p()
    arr = _tune_boxes()
    missing = str(tmp_path / "none.jsonl").encode()
    assert L.z4c_plan_create(arr, 1, ctypes.byref(p), None, missing, ctypes.byref(h)) == z4c.OK
    t, src = z4c.Tile(), ctypes.c_int()
    assert L.z4c_plan_tile(h, ctypes.byref(t), ctypes.byref(src)) == z4c.OK
    assert src.value == z4c.TILE_DEFAULT and t.persistent == 1
    assert L.z4c_plan_destroy(h) == z4c.OK
    bad = tmp_path / "bad.jsonl"
    bad.write_text("{broken\n")
    assert L.z4c_plan_create(arr, 1, ctypes.byref(p), None, str(bad).encode(), ctypes.byref(h)) == z4c.EINVAL
    assert b"tune cache" in L.z4c_last_error()
    # a caller tile wins over the cache and is reported as such
    t0 = z4c.tiles(z4c.FP64)[0]
    assert L.z4c_plan_create(arr, 1, ctypes.byref(p), ctypes.byref(t0), str(bad).encode(), ctypes.byref(h)) == z4c.OK
    assert L.z4c_plan_tile(h, ctypes.byref(t), ctypes.byref(src)) == z4c.OK
    assert src.value == z4c.TILE_CALLER and t.as_tuple()[:4] == t0.as_tuple()[:4]
    assert L.z4c_plan_destroy(h) == z4c.OK


def test_autotune_validation(L, tmp_path):
    p = z4c.default_params()
    arr = _tune_boxes()
    best, src = z4c.Tile(), ctypes.c_int()
    assert L.z4c_autotune(arr, 0, ctypes.byref(p), None, None, ctypes.byref(best), ctypes.byref(src)) == z4c.EINVAL
    assert L.z4c_autotune(arr, 1, None, None, None, ctypes.byref(best), ctypes.byref(src)) == z4c.EINVAL
    bad = tmp_path / "bad.jsonl"
    bad.write_text("[1, 2]\n")
    assert L.z4c_autotune(arr, 1, ctypes.byref(p), str(bad).encode(), None, ctypes.byref(best),
                          ctypes.byref(src)) == z4c.EINVAL
    assert bad.read_text() == "[1, 2]\n"  # a corrupt cache is left as it is


def test_strerror(L):
    for s in (z4c.OK, z4c.EINVAL, z4c.EHIP, z4c.ENOMEM, z4c.EUNSUPPORTED):
        assert len(L.z4c_strerror(s)) > 0


def test_product_path_has_no_oracle_dependency():
    """The package never imports the test oracle (it must fail loudly rather
    than fall back to a CPU path)."""
    pkg = os.path.dirname(z4c.__file__)
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(root, f)).read()
                assert "import oracle" not in text and "from oracle" not in text and "oz_" not in text, f


def test_library_shares_torch_hip_runtime():
    """Loading the library first (default_params before any torch import)
    still leaves one HIP runtime in the process: torch's, which owns the
    device memory and the streams handed to the library."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2607_08743_amd import z4c\n"
            "assert 'torch' not in sys.modules\n"
            "z4c.default_params()\n"
            "import torch, os\n"
            "libs = {os.path.realpath(l.split()[-1]) for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "tl = os.path.realpath(os.path.join(os.path.dirname(torch.__file__), 'lib'))\n"
            "print(len(libs), all(l.startswith(tl) for l in libs))\n") % root
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split()[-2:] == ["1", "True"], out.stdout


def test_constraints_workspace_size(L):
    # one partial per 8x8x4 brick of the active box, four constraints each
    assert L.z4c_constraints_workspace(256, 256, 256) == 4 * 32 * 32 * 64
    assert L.z4c_constraints_workspace(9, 8, 9) == 4 * 2 * 1 * 3
    assert L.z4c_constraints_workspace(0, 8, 8) == 0


def _cons(L, u=FAKE, c=None, norms=ctypes.c_void_p(0x20000000), ws=ctypes.c_void_p(0x30000000), ws_len=None,
          sf=12 ** 3, n=(6, 6, 6), ng=3, h=(0.1, 0.1, 0.1)):
    if ws_len is None:
        ws_len = L.z4c_constraints_workspace(*n)
    return L.z4c_constraints(u, c, norms, ws, ws_len, sf, n[0], n[1], n[2], ng, h[0], h[1], h[2], None)


@pytest.mark.parametrize("case", ["null_u", "null_norms", "null_ws", "small_ws", "ng2", "sf", "dx", "c_alias",
                                  "ws_alias", "norms_alias"])
def test_constraints_validation(L, case):
    kw = {}
    if case == "null_u":
        kw["u"] = None
    elif case == "null_norms":
        kw["norms"] = None
    elif case == "null_ws":
        kw["ws"] = None
    elif case == "small_ws":
        kw["ws_len"] = L.z4c_constraints_workspace(6, 6, 6) - 1
    elif case == "ng2":
        kw["ng"] = 2
    elif case == "sf":
        kw["sf"] = 12 ** 3 - 1
    elif case == "dx":
        kw["h"] = (0.1, 0.0, 0.1)
    elif case == "c_alias":
        kw["c"] = ctypes.c_void_p(0x10000 + 8 * 12 ** 3 * 24)   # inside u's 25 fields
    elif case == "ws_alias":
        kw["ws"] = ctypes.c_void_p(0x10000 + 8)
    elif case == "norms_alias":
        kw["norms"] = ctypes.c_void_p(0x10000 + 16)
    assert _cons(L, **kw) == z4c.EINVAL
    assert L.z4c_last_error().decode()


def test_equatorial_ghosts_reject_shell(L):
    # an equatorial box fills its mirrored layers itself: a shell is an error
    assert L.apply_ghosts(FAKE, FAKE2, 12 ** 3, 6, 6, 6, 3, z4c.BC_EQUATORIAL, None) == z4c.EINVAL
    assert "shell" in L.z4c_last_error().decode()


def _level(n=16, dx=1.0, x0=None, F=(4, 4, 4), bc=2, base=0x100000, parent=0, obj=-1):
    L = z4c.Level()
    L.n[:] = [n] * 3
    L.ng, L.bc = 3, bc
    L.sf = (n + 6) ** 3
    L.dx[:] = [dx] * 3
    L.x0[:] = [x0 if x0 is not None else -0.5 * (n - 1) * dx] * 3
    L.F[:] = list(F)
    size = 25 * L.sf * 8
    L.u, L.u_a, L.u_b, L.acc, L.prev, L.cur = [base + k * size for k in range(6)]
    L.parent, L.obj = parent, obj
    return L


HIER_CASES = {
    "dx": "dx must be half", "x0": "x0 does not put", "stencil": "prolongation stencil", "odd": "even",
    "bc0": "own boundary", "bc1": "Z4C_BC_COPY", "null": "six state arrays", "root_parent": "parent -1",
    "parent_order": "listed before", "root_moves": "cannot move", "shared": "overlap those of patch",
    "obj": "obj must be",
}


def test_hierarchy_adjacent_patches_accepted(L):
    """A small patch's arrays right before a larger patch's are not an
    overlap (each array spans its own field stride), although they lie
    within one large array's length of them."""
    n = 16
    base = 0x10000000
    parent = _level(n, 1.0, bc=z4c.BC_SOMMERFELD, parent=-1, base=base)
    x0c = -0.5 * (n - 1) * 1.0 + (4 - 0.25) * 1.0
    small = (n - 8 + 6) ** 3
    child = _level(n - 8, 0.5, x0=x0c, base=base - 6 * 25 * small * 8)
    arr = (z4c.Level * 2)(parent, child)
    h = ctypes.c_void_p()
    p = z4c.default_params()
    L.z4c_hier_create(arr, 2, ctypes.byref(p), 0.5, None, ctypes.byref(h))
    assert "overlap" not in L.z4c_last_error().decode()


@pytest.mark.parametrize("case", sorted(HIER_CASES))
def test_hierarchy_validation(L, case):
    """z4c_hier_create rejects inconsistent patch geometry and links before
    it would touch the GPU, each with its own message."""
    n = 16
    parent = _level(n, 1.0, bc=z4c.BC_SOMMERFELD, parent=-1)
    x0c = -0.5 * (n - 1) * 1.0 + (4 - 0.25) * 1.0
    child = _level(n, 0.5, x0=x0c, base=0x800000000)
    if case == "dx":
        child.dx[:] = [0.4] * 3
    elif case == "x0":
        child.x0[:] = [x0c + 0.1] * 3
    elif case == "stencil":
        child.F[:] = [1, 4, 4]
        child.x0[0] = -0.5 * (n - 1) + (1 - 0.25)
    elif case == "odd":
        child.n[:] = [15, 16, 16]
    elif case == "bc0":
        parent.bc = z4c.BC_COPY
    elif case == "bc1":
        child.bc = z4c.BC_PERIODIC
    elif case == "null":
        child.cur = None
    elif case == "root_parent":
        parent.parent = 0
    elif case == "parent_order":
        child.parent = 1
    elif case == "root_moves":
        parent.obj = 0
    elif case == "shared":
        child.prev = parent.u + 8  # inside the parent's state
    elif case == "obj":
        child.obj = -2
    arr = (z4c.Level * 2)(parent, child)
    h = ctypes.c_void_p()
    p = z4c.default_params()
    assert L.z4c_hier_create(arr, 2, ctypes.byref(p), 0.5, None, ctypes.byref(h)) == z4c.EINVAL
    assert HIER_CASES[case] in L.z4c_last_error().decode(), L.z4c_last_error().decode()
    assert not h.value


def test_size_limits(L):
    """Offsets inside one field are 32-bit in the kernels: a box of more than
    2^31 - 1 stored points per field, or an extent above 2^20, is refused; the
    largest cube under the limit passes the geometry check (the call then
    fails on its NULL state pointer, after it)."""
    p = z4c.default_params()
    assert _rhs(L, p, sf=1 << 40, n=(1285, 1285, 1285)) == z4c.EINVAL  # 1291^3 > 2^31 - 1
    assert "2^31-1" in L.z4c_last_error().decode()
    assert _rhs(L, p, sf=1 << 40, n=(1 << 20, 1, 1)) == z4c.EINVAL
    assert "extent too large" in L.z4c_last_error().decode()
    assert 1290 ** 3 <= (1 << 31) - 1
    assert _rhs(L, p, u=None, sf=1290 ** 3, n=(1284, 1284, 1284)) == z4c.EINVAL
    msg = L.z4c_last_error().decode()
    assert "stored points" not in msg and "extent" not in msg, msg


def test_missing_library_fails_loudly():
    """Without the built library the binding raises on every call: there is
    no CPU fallback behind the product path."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2607_08743_amd import z4c\n"
            "z4c.lib.__defaults__ = ('/nonexistent/libz4c.so',)\n"
            "for call in (lambda: z4c.lib(), lambda: z4c.default_params()):\n"
            "    try:\n"
            "        call()\n"
            "        print('no error')\n"
            "    except RuntimeError as e:\n"
            "        print('raised', 'not built' in str(e))\n") % root
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["raised", "True", "raised", "True"], out.stdout


def test_constraints_noalloc_validation(L):
    """The allocation-free monitor refuses boxes beyond its fixed array (more
    than Z4C_CONSTRAINTS_NOALLOC_MAX_BLOCKS bricks of 8x8x4) and bad arguments
    before any HIP call."""
    n = 520  # 65 x 65 x 130 = 549250 bricks > 524288
    sf = (n + 6) ** 3
    args = (sf, n, n, n, 3, 0.1, 0.1, 0.1, None)
    assert L.z4c_constraints_noalloc(FAKE, None, FAKE2, *args) == z4c.EINVAL
    assert b"too large" in L.z4c_last_error()
    assert L.z4c_constraints_noalloc(None, None, FAKE2, 14 ** 3, 8, 8, 8, 3, 0.1, 0.1, 0.1, None) == z4c.EINVAL
    assert L.z4c_constraints_noalloc(FAKE, None, None, 14 ** 3, 8, 8, 8, 3, 0.1, 0.1, 0.1, None) == z4c.EINVAL
    assert L.z4c_constraints_noalloc(FAKE, None, FAKE2, 14 ** 3, 8, 8, 8, 2, 0.1, 0.1, 0.1, None) == z4c.EINVAL
