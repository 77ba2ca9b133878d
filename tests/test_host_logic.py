"""Host-side checks of the HIP library that need no GPU: the C ABI exports,
the lattice builder, the pass planner and, by a CPU re-enactment of the
kernels' index arithmetic, that every pass touches each amplitude exactly
once and stays inside its buffers (state, LDS, phase table, partials)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2108_13410_amd import z2h

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LDS_LIMIT = 160 * 1024


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "z2h.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(z2h_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_header_symbol():
    L = ctypes.CDLL(z2h.LIB_PATH)
    syms = header_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) <= set(z2h.SIGNATURES), set(syms) - set(z2h.SIGNATURES)
    assert z2h.z2h_version().startswith("z2h")


@pytest.mark.parametrize("Lx,Ly", [(2, 2), (2, 3), (3, 3), (3, 4), (4, 4), (2, 8)])
def test_library_lattice(Lx, Ly):
    """Library numbering: stars/plaquettes of four links, each link on two of
    each, even star-plaquette overlaps, products of all stars (plaquettes) = I."""
    st, pl = z2h.z2h_masks(Lx, Ly)
    n = 2 * Lx * Ly
    seen = set()
    for y in range(Ly):
        for x in range(Lx):
            for d in (0, 1):
                seen.add(z2h.z2h_link_bit(Lx, Ly, x, y, d))
    assert seen == set(range(n))
    for m in list(st) + list(pl):
        assert bin(int(m)).count("1") == 4
    for l in range(n):
        assert sum(int(m) >> l & 1 for m in st) == 2
        assert sum(int(m) >> l & 1 for m in pl) == 2
    for a in st:
        for b in pl:
            assert bin(int(a) & int(b)).count("1") % 2 == 0
    xs = xp = 0
    for a, b in zip(st, pl):
        xs ^= int(a)
        xp ^= int(b)
    assert xs == 0 and xp == 0


def test_invalid_arguments_rejected_without_gpu():
    with pytest.raises(z2h.Z2HError) as e:
        z2h.z2h_plan_create(1, 3, z2h.Z2H_C64)
    assert e.value.code == z2h.Z2H_ERR_INVALID
    with pytest.raises(z2h.Z2HError) as e:
        z2h.z2h_plan_create(4, 5, z2h.Z2H_C64)
    assert e.value.code == z2h.Z2H_ERR_UNSUPPORTED
    with pytest.raises(z2h.Z2HError):
        z2h.z2h_plan_create(3, 3, 7)
    with pytest.raises(z2h.Z2HError):
        z2h.z2h_plan_create(3, 3, z2h.Z2H_C64, 20)
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C64)
    L = z2h.lib()
    s = z2h.schedule((1, 1, 0, 0), (1, 1, .3, .3), 10, 0.1)
    # null state / workspace, misaligned state, bad step range, bad dt
    assert L.z2h_evolve(plan.handle, None, ctypes.c_void_p(4096), 1 << 20, ctypes.byref(s), None, None) == z2h.Z2H_ERR_INVALID
    assert L.z2h_evolve(plan.handle, ctypes.c_void_p(4096 + 8), ctypes.c_void_p(4096), 1 << 20, ctypes.byref(s), None, None) == z2h.Z2H_ERR_INVALID
    assert L.z2h_evolve(plan.handle, ctypes.c_void_p(4096), None, 1 << 20, ctypes.byref(s), None, None) == z2h.Z2H_ERR_INVALID
    assert L.z2h_evolve(plan.handle, ctypes.c_void_p(4096), ctypes.c_void_p(8192), 8, ctypes.byref(s), None, None) == z2h.Z2H_ERR_WORKSPACE
    bad = z2h.schedule((1, 1, 0, 0), (1, 1, .3, .3), 10, 0.1, k_begin=5, k_end=3)
    assert L.z2h_evolve(plan.handle, ctypes.c_void_p(4096), ctypes.c_void_p(8192), 1 << 20, ctypes.byref(bad), None, None) == z2h.Z2H_ERR_INVALID
    bad = z2h.schedule((1, 1, 0, 0), (1, 1, .3, .3), 10, float("nan"))
    assert L.z2h_evolve(plan.handle, ctypes.c_void_p(4096), ctypes.c_void_p(8192), 1 << 20, ctypes.byref(bad), None, None) == z2h.Z2H_ERR_INVALID
    bad = z2h.schedule((1, 1, 0, 0), (1, 1, .3, .3), 10, 0.1, order=2)
    assert L.z2h_evolve(plan.handle, ctypes.c_void_p(4096), ctypes.c_void_p(8192), 1 << 20, ctypes.byref(bad), None, None) == z2h.Z2H_ERR_INVALID
    bad = z2h.schedule((1, 1, 0, 0), (1, 1, .3, .3), 3, 0.1, sZ=[0.1, float("inf"), 0.2])
    assert L.z2h_evolve(plan.handle, ctypes.c_void_p(4096), ctypes.c_void_p(8192), 1 << 20, ctypes.byref(bad), None, None) == z2h.Z2H_ERR_INVALID
    H = z2h.couplings(1, 1, .3, .3)
    big = (ctypes.c_uint64 * 1)(1 << 40)
    assert L.z2h_observe(plan.handle, ctypes.c_void_p(4096), ctypes.c_void_p(8192), 1 << 30, ctypes.byref(H), big, 1, None, 0, None, ctypes.c_void_p(4096), None) == z2h.Z2H_ERR_INVALID
    assert L.z2h_observe(plan.handle, ctypes.c_void_p(4096), ctypes.c_void_p(8192), 1 << 30, ctypes.byref(H), None, 9, None, 0, None, ctypes.c_void_p(4096), None) == z2h.Z2H_ERR_INVALID
    assert L.z2h_observe(plan.handle, ctypes.c_void_p(4096), ctypes.c_void_p(8192), 16, ctypes.byref(H), None, 0, None, 0, None, ctypes.c_void_p(4096), None) == z2h.Z2H_ERR_WORKSPACE
    assert L.z2h_state_init(plan.handle, ctypes.c_void_p(4096), 9, None) == z2h.Z2H_ERR_INVALID
    assert "init kind" in z2h.z2h_last_error()


# ------------------------------------------------------------------ planner re-enactment

def lay_base(p, t, R):
    return (t & ((1 << p) - 1)) | ((t >> p) << (p + R))


def local_positions(g):
    """Global bit of each local tile bit: carried bits [0, c), then the run
    at b0, then (split groups, hi > 0) the run of hi bits at b1."""
    c, b0, m, hi = g["c"], g["b0"], g["m"], g.get("hi", 0)
    ga = m - c - hi
    return list(range(c)) + list(range(b0, b0 + ga)) + list(range(g.get("b1", 0), g.get("b1", 0) + hi))


def tile_positions(g, n):
    """Global bits of the tile index: every other bit, ascending."""
    loc = set(local_positions(g))
    return [b for b in range(n) if b not in loc]


def deposit(v, positions):
    v = np.asarray(v, dtype=np.int64)
    out = np.zeros_like(v)
    for i, pos in enumerate(positions):
        out |= ((v >> i) & 1) << pos
    return out


def glob(g, tile, e, n=None):
    n = n if n is not None else g["tiles_log2"] + g["m"]
    return deposit(e, local_positions(g)) | deposit(tile, tile_positions(g, n))


def gbit(g, x):
    return local_positions(g)[x]


PLANS = [(2, 2, 0, 0), (2, 2, 1, 0), (2, 3, 0, 0), (2, 3, 1, 0), (3, 3, 0, 0), (3, 3, 1, 0),
         (3, 3, 0, 8), (3, 3, 1, 8), (3, 3, 1, 10), (3, 3, 0, 9), (2, 4, 0, 0), (3, 2, 1, 0),
         (3, 4, 0, 0), (3, 4, 1, 0), (2, 7, 1, 0), (4, 4, 0, 0), (4, 4, 1, 0)]


@pytest.mark.parametrize("Lx,Ly,dt,mtb", PLANS)
def test_pass_geometry(Lx, Ly, dt, mtb):
    check_geometry(z2h.z2h_plan_create(Lx, Ly, dt, mtb))


@pytest.mark.parametrize("Lx,Ly,dt", [(3, 3, 0), (3, 3, 1), (3, 4, 0), (4, 4, 0), (4, 4, 1)])
def test_autotuner_candidates_are_valid_plans(Lx, Ly, dt):
    """Every schedule the autotuner may pick builds a plan whose passes cover
    each amplitude once and stay inside their buffers."""
    cands = z2h.z2h_tune_candidates(Lx, Ly, dt)
    assert len(cands) >= 4
    for c in cands:
        check_geometry(z2h.z2h_plan_create_config(Lx, Ly, dt, c))


def test_shipped_schedules_are_candidates():
    """The shipped table's schedules build valid plans, and the 4x4 ones
    (groups in two runs of qubits) are among the autotuner's candidates."""
    import os
    table = os.path.join(os.path.dirname(z2h.__file__), "tuned_mi355x.txt")
    rows = [l.split() for l in open(table) if l.strip() and not l.startswith("#")]
    assert rows
    for n, c128, _bc, cfg in rows:
        Lx, Ly = {18: (3, 3), 32: (4, 4)}[int(n)]
        dt = z2h.Z2H_C128 if int(c128) else z2h.Z2H_C64
        check_geometry(z2h.z2h_plan_create_config(Lx, Ly, dt, cfg))
        if int(n) == 32:
            assert cfg in z2h.z2h_tune_candidates(Lx, Ly, dt), cfg


def test_block_order_option():
    """Group 0 runs in XCD-major block order by default; ",xcd=<mask>"
    selects the groups (bits above the group count are dropped)."""
    d = z2h.z2h_plan_describe(z2h.z2h_plan_create(3, 3, z2h.Z2H_C64))
    assert d["xcd"] == 1
    for cfg, want in (("split=12:4:12:0/6:3:11:5:2", 1), ("split=12:4:12:0/6:3:11:5:2,xcd=0", 0),
                      ("split=12:4:12:0/6:3:11:5:2,xcd=3", 3), ("uniform,m=12,c=4,xcd=2", 2),
                      ("split=12:4:12:0/6:3:11:5:2,xcd=255", 15), ("split=12:4:12:0/6:3:11:5:2,nt=1,xcd=0", 0)):
        d = z2h.z2h_plan_describe(z2h.z2h_plan_create_config(3, 3, z2h.Z2H_C64, cfg))
        assert d["xcd"] == want, cfg
    assert z2h.z2h_plan_describe(z2h.z2h_plan_create_config(3, 3, z2h.Z2H_C64, "uniform,m=12,nt=1"))["nt"] == 1


def test_schedule_strings_rejected():
    for bad in ("split=10:5:13:0", "split=10:5:13:1/8:4:13:5", "split=10:5:13:0/8:4:19:11", "split=10:5:16:0/8:4:13:5",
                "split=10:5:11:0/8:4:13:5:3", "split=18:3:18:0:2", "nonsense"):
        with pytest.raises(z2h.Z2HError):
            z2h.z2h_plan_create_config(3, 3, z2h.Z2H_C64, bad)
    # two-tile blocks exist for complex64 only
    with pytest.raises(z2h.Z2HError):
        z2h.z2h_plan_create_config(3, 3, z2h.Z2H_C128, "split=12:4:12:0/6:3:10:4:2")
    ok = z2h.z2h_plan_create_config(3, 3, z2h.Z2H_C64, "split=10:5:11:0/8:4:12:4:2")
    assert z2h.z2h_plan_describe(ok)["groups"][1]["pair"] == 2
    check_geometry(ok)
    # component exchange: one tile per block, shapes with a compiled kernel
    for dt, cfg in ((z2h.Z2H_C64, "split=10:5:11:0:1c/10:5:14:4:1c"), (z2h.Z2H_C128, "split=10:5:11:0/10:5:13:3:1c")):
        cp = z2h.z2h_plan_create_config(2, 5, dt, cfg)
        d = z2h.z2h_plan_describe(cp)
        assert [g["cx"] for g in d["groups"]] == ([1, 1] if dt == z2h.Z2H_C64 else [0, 1])
        full = z2h.z2h_plan_describe(z2h.z2h_plan_create_config(2, 5, dt, cfg.replace(":1c", "")))
        assert d["groups"][1]["lds_bytes"] < 0.6 * full["groups"][1]["lds_bytes"]
        check_geometry(cp)
    for bad in ("split=10:5:11:0:2c/10:5:14:4", "split=10:5:11:0:3/10:5:14:4"):
        with pytest.raises(z2h.Z2HError):
            z2h.z2h_plan_create_config(2, 5, z2h.Z2H_C64, bad)
    with pytest.raises(z2h.Z2HError):  # window shape without a component-exchange kernel
        z2h.z2h_plan_create_config(3, 3, z2h.Z2H_C64, "split=12:4:12:0/6:3:11:5:1c")
    # group 0 in two-tile blocks (two adjacent chunks)
    ok0 = z2h.z2h_plan_create_config(3, 3, z2h.Z2H_C64, "split=12:4:12:0:2/6:3:11:5:2")
    assert [g["pair"] for g in z2h.z2h_plan_describe(ok0)["groups"]] == [2, 2]
    check_geometry(ok0)


def test_split_run_groups():
    """":h<N>": a strided group takes its top N bits from the top of the
    state (two runs of global bits); later groups continue below them."""
    cfg = "split=12:4:12:0/10:5:14:4:1c:h5/10:5:14:4:1c,xcd=7"
    d = z2h.z2h_plan_describe(z2h.z2h_plan_create_config(4, 4, z2h.Z2H_C64, cfg))
    g1, g2 = d["groups"][1], d["groups"][2]
    assert (g1["b0"], g1["hi"], g1["b1"]) == (12, 5, 27)
    assert (g2["b0"], g2["hi"]) == (17, 0)
    assert gbit(g1, 4) == 12 and gbit(g1, 8) == 16 and gbit(g1, 9) == 27 and gbit(g1, 13) == 31
    check_geometry(z2h.z2h_plan_create_config(4, 4, z2h.Z2H_C64, cfg))
    check_geometry(z2h.z2h_plan_create_config(4, 4, z2h.Z2H_C128, "split=12:4:12:0/10:5:13:3:1c:h5/10:5:13:3:1c"))
    # explicit run positions; the last group takes the free qubits, here in two runs
    for dt, cfg, want in (
            (z2h.Z2H_C64, "split=12:4:12:0/10:5:14:4:1c:h5@23/10:5:14:4:1c", [(12, 5, 23), (17, 4, 28)]),
            (z2h.Z2H_C128, "split=12:4:12:0/10:5:13:3:1c:h7@22/10:5:13:3:1c", [(12, 7, 22), (15, 3, 29)]),
            (z2h.Z2H_C64, "split=12:4:12:0/10:5:14:4:1c:at17:h4@28/10:5:14:4:1c", [(17, 4, 28), (12, 5, 23)])):
        plan = z2h.z2h_plan_create_config(4, 4, dt, cfg)
        gs = z2h.z2h_plan_describe(plan)["groups"]
        assert [(g["b0"], g["hi"], g["b1"]) for g in gs[1:]] == want, cfg
        check_geometry(plan)
    # small enough for the exhaustive tile-coverage check (n = 20): a window
    # across the two runs in the middle group, and in the last (phase) group
    for dt, cfg, j, want in ((z2h.Z2H_C64, "split=4:2:8:0/10:5:14:4:1c:h3@17/6:3:10:4", 1, (4, 3, 17)),
                             (z2h.Z2H_C128, "split=4:2:8:0/10:5:13:3:1c:h3@17/6:3:9:3", 1, (4, 3, 17)),
                             (z2h.Z2H_C64, "split=4:2:8:0/6:3:10:4:at8/10:5:14:4:1c", 2, (4, 6, 14)),
                             (z2h.Z2H_C128, "split=4:2:8:0/6:3:9:3:at8/10:5:13:3:1c", 2, (4, 6, 14))):
        if True:
            small = z2h.z2h_plan_create_config(2, 5, dt, cfg)
            gj = z2h.z2h_plan_describe(small)["groups"][j]
            assert (gj["b0"], gj["hi"], gj["b1"]) == want
            check_geometry(small)
    for bad in ("split=12:4:12:0:h4/10:5:14:4/10:5:14:4",         # group 0 cannot split
                "split=12:4:12:0/10:5:14:4:h3/10:5:14:4",           # two runs without :1c
                "split=12:4:12:0/10:5:14:4:h5/10:5:14:4",           # two runs without :1c
                "split=12:4:12:0/10:5:14:4:h10/10:5:14:4",          # high run as wide as the group
                "split=12:4:12:0/10:5:14:4:h5/10:5:14:4/5:5:9:4",   # covers more than n bits
                "split=12:4:12:0/10:5:14:4:1c:h5@14/10:5:14:4:1c",  # runs overlap
                "split=12:4:12:0/10:5:14:4:1c:at10/10:5:14:4:1c",   # qubits of group 0
                "split=12:4:12:0/10:5:14:4:1c:h5@30/10:5:14:4:1c",  # past the last qubit
                "split=12:4:12:0/10:5:14:4:hx/10:5:14:4"):
        with pytest.raises(z2h.Z2HError):
            z2h.z2h_plan_create_config(4, 4, z2h.Z2H_C64, bad)
    # groups that are not whole windows (general pass kernel) may take two runs too
    for dt, cfg in ((z2h.Z2H_C128, "split=12:4:12:0/10:4:13:3:h7@22/10:4:13:3"),
                    (z2h.Z2H_C64, "split=4:2:8:0/10:4:13:3:h3@17/6:3:10:4")):
        plan = z2h.z2h_plan_create_config(4 if dt == z2h.Z2H_C128 else 2, 4 if dt == z2h.Z2H_C128 else 5, dt, cfg)
        gs = z2h.z2h_plan_describe(plan)["groups"]
        assert gs[1]["hi"] and not gs[1]["full"]
        check_geometry(plan)
    # complex128 tiles of 2^14 amplitudes: the passes fit (component
    # exchange), the observables' whole-element transform does not
    with pytest.raises(z2h.Z2HError):
        z2h.z2h_plan_create_config(2, 5, z2h.Z2H_C128, "split=4:2:8:0/10:5:14:4:1c:h3@17/6:3:10:4")


def check_full_lds(g, n, esize):
    """Re-enact the full-window kernels' LDS placement: one slot per local
    index inside the allocated block, and the bank pattern of every layout
    change (each group of 2^lb consecutive lanes of a wave, 2^lb = 256 bytes /
    element size, for both the writes and the reads)."""
    R, NL, m, c, x0, x1 = g["R"], g["full"], g["m"], g["c"], g["x0"], g["x1"]
    G = R * NL
    blk = g["lds_blk"]
    assert blk >= (1 << G) + (1 << (G - R))
    ex = esize // 2 if g.get("cx") else esize  # bytes per LDS slot (component exchange: one component)
    lb = {4: 6, 8: 5, 16: 4}[ex]

    def place(e):
        tb = (e >> x0) & ((1 << G) - 1)
        u = (e & ((1 << x0) - 1)) | ((e >> x1) << x0)
        return tb + (tb >> R) + u * blk

    e = np.arange(1 << m)
    a = place(e)
    assert np.unique(a).size == e.size
    assert a.max() < (1 << (m - G)) * blk
    assert (1 << (m - G)) * blk * ex + (n // 2 + 1) * (n + 1) * esize <= LDS_LIMIT
    assert g["lds_bytes"] <= LDS_LIMIT
    threads = 1 << (m - R)
    t = np.arange(threads)
    for j in range(NL):
        p = x1 - R * (j + 1)
        base = place(lay_base(p, t, R))
        for q in range(1 << R):
            addr = base + (q << (G - R * (j + 1))) + ((q << (G - R * (j + 1))) >> R)
            # the compile-time offset form equals the direct placement
            assert np.array_equal(addr, place(lay_base(p, t, R) | (q << p)))
            for w0 in range(0, min(threads, 64), 1 << lb):
                grp = addr[w0:w0 + (1 << lb)] % (1 << lb)
                worst = np.bincount(grp).max()
                # conflict-free, except that contiguous groups with narrow
                # windows keep the transform padding's at most 2-way overlap
                assert worst <= (1 if c > 0 else 2), (g, j, q, w0, worst)


def check_geometry(plan):
    d = z2h.z2h_plan_describe(plan)
    n, K = d["n"], d["K"]
    assert K == len(d["groups"])
    covered = []
    for gi, g in enumerate(d["groups"]):
        R = g["R"]
        m, c, b0, x0, x1 = g["m"], g["c"], g["b0"], g["x0"], g["x1"]
        if g["full"]:
            # straight-line kernels: NL complete windows at x1 - R (j + 1)
            assert (x1 - x0) == g["full"] * R
            assert g["p"] == [x1 - R * (j + 1) for j in range(g["full"])]
        threads = 1 << (m - R)
        assert 64 <= threads <= 512
        assert g["lds_bytes"] <= LDS_LIMIT
        assert g["tiles_log2"] == n - m
        # local bits [0,c) and [c,m) map to global [0,c) and [b0, b0+m-c)
        # (split groups: [b0, b0+m-c-hi) and [b1, b1+hi)); tile bits fill the rest
        hr = g["hi"]
        local = set(local_positions(g))
        assert len(local) == m and local == set(range(c)) | set(range(b0, b0 + m - c - hr)) | set(
            range(g["b1"], g["b1"] + hr))
        tilebits = set(tile_positions(g, n))
        assert not (local & tilebits) and (local | tilebits) == set(range(n))
        if hr:
            # two separate runs: groups of whole windows only with the
            # component exchange (the other straight-line kernels keep one run)
            assert g["b1"] > b0 + m - c - hr
            assert not g["full"] or g["cx"] == 1
        covered += [gbit(g, x) for x in range(x0, x1)]
        # layouts: windows of R local bits inside the transform range, never
        # straddling the carried boundary; butterflies cover [x0, x1) once
        done = set()
        for p, lo, hi in zip(g["p"], g["blo"], g["bhi"]):
            assert x0 <= p and p + R <= m
            assert p >= c or p + R <= c
            bits = set(range(p + lo, p + hi))
            assert bits <= set(range(x0, x1)) and not (bits & done)
            done |= bits
        assert done == set(range(x0, x1))
        # every layout maps (thread, q) onto the 2^m local indices exactly once,
        # and the LDS slot stays inside the padded buffer
        t = np.arange(threads)
        for p in g["p"]:
            e = np.concatenate([lay_base(p, t, R) | (q << p) for q in range(1 << R)])
            assert np.array_equal(np.sort(e), np.arange(1 << m))
            slot = e + (e >> R)
            assert slot.max() < (1 << m) + (1 << (m - R))
            # register bits as the kernels place them: [gs, gs + nlo), then
            # (a window across the two runs of a split group) [b1, ...)
            gs = gbit(g, p)
            xb = m - hr
            nlo = xb - p if hr and p < xb < p + R else R
            P = [gs + r if r < nlo else g["b1"] + r - nlo for r in range(R)]
            assert P == [gbit(g, p + r) for r in range(R)]
            # register element q is at global index i0 + reg_off(q)
            for q in (1, (1 << R) - 1, (1 << R) // 2 + 1):
                off = sum(1 << P[r] for r in range(R) if q >> r & 1)
                for tile in (0, (1 << g["tiles_log2"]) - 1):
                    i_direct = glob(g, tile, lay_base(p, t, R) | (q << p))
                    i_split = glob(g, tile, lay_base(p, t, R)) + off
                    assert np.array_equal(i_direct, i_split)
                    assert i_direct.max() < (1 << n)
        if g["full"] and K > 1:
            check_full_lds(g, n, 16 if d["c128"] else 8)
        if g.get("pair", 1) == 2:
            # two-tile blocks: tiles 2u and 2u + 1 differ only in global bit c
            # (a strided group's rows become 2^(c+1) contiguous amplitudes) or,
            # in group 0, in bit m (two adjacent chunks of 2^m amplitudes)
            assert g["tiles_log2"] >= 1 and g["full"]
            assert (gi > 0 and b0 - c >= 1) or (gi == 0 and c == 0)
            step = 1 << c if gi > 0 else 1 << m
            e = np.arange(1 << m)
            for u in (0, (1 << (g["tiles_log2"] - 1)) - 1):
                assert np.array_equal(glob(g, 2 * u + 1, e) - glob(g, 2 * u, e), np.full(e.size, step))
        if n <= 20:
            # all tiles together cover the state exactly once
            e = np.arange(1 << m)
            tiles = np.arange(1 << g["tiles_log2"])
            allidx = (glob(g, tiles, 0, n)[:, None] | glob(g, 0, e, n)[None, :]).ravel()
            assert np.array_equal(np.sort(allidx), np.arange(1 << n))
    assert sorted(covered) == list(range(n))
    # phase table: index popc(syndrome) * (n + 1) + w stays below (nst + 1)(n + 1)
    nst = n // 2
    assert nst * (n + 1) + n < (nst + 1) * (n + 1)


def test_level_sequence_counts():
    """Levels per ramp: x-z-x visits the outer group S+1 times and the inner
    group S times with a phase; every step's phases appear exactly once."""
    for K in (2, 3, 4):
        for S in (1, 2, 5):
            plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C64, {2: 0, 3: 10, 4: 8}[K])
            assert z2h.z2h_plan_info(plan)["groups"] == K
            info = z2h.z2h_plan_info(plan)
            assert info["passes_per_step"] == 2 * (K - 1)


@pytest.mark.parametrize("Lx,Ly", [(2, 2), (3, 3), (3, 4), (4, 4)])
def test_loop_masks(Lx, Ly):
    """The reported loops: the strip and L loops are products of plaquettes
    (contractible, commute with every star); W1, W2 and V1, V2 are the
    noncontractible pairs (V1 anticommutes with W2, V2 with W1)."""
    import oracle
    zl, xl = z2h.z2h_loop_masks(Lx, Ly)
    st, pl = z2h.z2h_masks(Lx, Ly)
    strip = 0
    for x in range(min(3, Lx)):
        strip ^= int(pl[x])
    assert zl[0] == strip
    assert zl[1] == int(pl[0]) ^ int(pl[1]) ^ int(pl[Lx])
    for m in zl:
        for a in st:
            assert bin(m & int(a)).count("1") % 2 == 0
    for m in xl:
        for b in pl:
            assert bin(m & int(b)).count("1") % 2 == 0
    assert bin(xl[0] & zl[3]).count("1") % 2 == 1
    assert bin(xl[1] & zl[2]).count("1") % 2 == 1
    # same loops as the oracle's, through the link-coordinate map
    from helpers import mask_lib_to_oracle
    ol = oracle.loops(Lx, Ly)
    assert mask_lib_to_oracle(Lx, Ly, zl[2]) == ol["W1"]
    assert mask_lib_to_oracle(Lx, Ly, zl[3]) == ol["W2"]
    assert mask_lib_to_oracle(Lx, Ly, xl[0]) == ol["V1"]
    assert mask_lib_to_oracle(Lx, Ly, xl[1]) == ol["V2"]


@pytest.mark.parametrize("tune", ["uniform,m=13,R=3,c=4", "uniform,m=14,R=2,c=4", "uniform,m=8,R=5,c=4", "uniform,m=12,R=2,c=3"])
def test_out_of_bounds_tunings_rejected(tune, monkeypatch):
    """Tile/register choices that would exceed the kernels' launch bounds
    (64..512 threads), the layout table or LDS are refused at plan creation."""
    monkeypatch.setenv("Z2H_TUNE", tune)
    with pytest.raises(z2h.Z2HError) as e:
        z2h.z2h_plan_create(3, 3, z2h.Z2H_C64)
    assert e.value.code == z2h.Z2H_ERR_UNSUPPORTED


def test_path_sample_count_and_validation():
    """Size query of z2h_path_evolve (no device work) and path validation."""
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C64)
    L = z2h.lib()
    ns = ctypes.c_int64()
    p = z2h.make_path([(1, 1, 0, 0), (1, 1, .2, 0), (1, 1, .2, .1), (1, 1, .2, .1)], [25, 0, 10], 0.02, every=10)
    assert L.z2h_path_evolve(plan.handle, None, None, 0, ctypes.byref(p), None, 0, None, 0, None, 0,
                             ctypes.byref(ns), None) == z2h.Z2H_OK
    assert ns.value == 1 + 3 + 0 + 1
    p0 = z2h.make_path([(1, 1, 0, 0), (1, 1, .2, 0)], [25], 0.02, every=0)
    assert L.z2h_path_evolve(plan.handle, None, None, 0, ctypes.byref(p0), None, 0, None, 0, None, 0,
                             ctypes.byref(ns), None) == z2h.Z2H_OK
    assert ns.value == 2
    bad = [z2h.make_path([(1, 1, 0, 0), (1, 1, .2, 0)], [-1], 0.02),
           z2h.make_path([(1, 1, 0, 0), (1, 1, float("nan"), 0)], [5], 0.02),
           z2h.make_path([(1, 1, 0, 0), (1, 1, .2, 0)], [5], 0.02, sampling=2),
           z2h.make_path([(1, 1, 0, 0), (1, 1, .2, 0)], [5], 0.02, every=-3)]
    for q in bad:
        assert L.z2h_path_evolve(plan.handle, None, None, 0, ctypes.byref(q), None, 0, None, 0, None, 0,
                                 ctypes.byref(ns), None) == z2h.Z2H_ERR_INVALID
    # a trace too small for the samples is a workspace error, raised before any device work
    assert L.z2h_path_evolve(plan.handle, ctypes.c_void_p(4096), ctypes.c_void_p(8192), 1 << 30,
                             ctypes.byref(p), None, 0, None, 0, ctypes.c_void_p(4096), 2,
                             ctypes.byref(ns), None) == z2h.Z2H_ERR_WORKSPACE


# ------------------------------------------------------------------ exact solvers (host parts)

def _tridiag(m, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=m) * 3.0, rng.uniform(0.05, 2.0, size=m - 1)


@pytest.mark.parametrize("m", [1, 2, 7, 40, 300])
def test_tridiag_lowest_against_eigvalsh(m):
    """Sturm bisection of the Lanczos matrix: the lowest eigenvalue equals
    numpy's dense symmetric eigensolver on the same tridiagonal matrix."""
    a, b = _tridiag(m, m)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    ref = np.linalg.eigvalsh(T)[0]
    got = z2h.z2h_tridiag_lowest(a, b)
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (got, ref)


def test_tridiag_lowest_degenerate_cases():
    """A split matrix (beta = 0) and a multiple eigenvalue."""
    a = np.array([3.0, -1.0, 2.0, -1.0])
    b = np.array([0.0, 0.0, 0.0])
    assert z2h.z2h_tridiag_lowest(a, b) == pytest.approx(-1.0, abs=1e-14)
    a, b = np.array([2.0, 2.0]), np.array([0.0])
    assert z2h.z2h_tridiag_lowest(a, b) == pytest.approx(2.0, abs=1e-14)


@pytest.mark.parametrize("m,tau", [(1, 0.3), (2, 0.7), (12, 0.02), (32, 0.5), (32, 3.0)])
def test_tridiag_expv_against_expm(m, tau):
    """exp(-i tau T) e_1 of the Krylov step equals scipy's dense expm."""
    import scipy.linalg as sla
    a, b = _tridiag(m, 100 + m)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    ref = sla.expm(-1j * tau * T)[:, 0]
    got = z2h.z2h_tridiag_expv(a, b, tau)
    assert np.abs(got - ref).max() < 1e-12


def test_exact_solver_sizes_and_argument_checks():
    """Workspace sizes (state-sized vectors plus coefficient records) and the
    rejections that happen before any device work."""
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    state = 16 << 18
    w_l = z2h.z2h_lanczos_sizes(plan, 100)
    assert 2 * state <= w_l < 2 * state + 128 * 1024
    w_e = z2h.z2h_exact_sizes(plan, 12)
    assert 13 * state <= w_e < 13 * state + 128 * 1024
    for bad in (0, 100001):
        with pytest.raises(z2h.Z2HError):
            z2h.z2h_lanczos_sizes(plan, bad)
    for bad in (0, 33):
        with pytest.raises(z2h.Z2HError):
            z2h.z2h_exact_sizes(plan, bad)
    with pytest.raises(z2h.Z2HError):
        z2h.lib()  # library loads; the call below fails on the NULL buffers
        code = z2h.lib().z2h_hamiltonian_apply(plan.handle, None, None, ctypes.byref(z2h.couplings()), None)
        z2h._check(code)
    with pytest.raises(z2h.Z2HError):
        z2h._check(z2h.lib().z2h_tridiag_expv(33, None, None, 0.1, None, None))


# ------------------------------------------------------------------ gate-level circuits (host parts)

@pytest.mark.parametrize("Lx,Ly", [(2, 2), (2, 3), (3, 3), (3, 4), (4, 4)])
def test_circuit_step_structure(Lx, Ly):
    """The library's step circuit: 3n field rotations and, in each of the two
    stabilizer halves, a CNOT-R_z-CNOT gadget per plaquette and the same
    inside Hadamards per star (3n + 52 Ns gates; 522 at 3x3).  Every CNOT
    targets the ancilla (qubit n), every R_z on the ancilla carries the
    coupling's angle, and the layers come in the order of Eq. (decom)."""
    n, nv = 2 * Lx * Ly, Lx * Ly
    cx, cz, dt = (0.7, 0.4, 0.3, 0.2), (0.6, 0.9, 0.1, 0.45), 0.37
    arr, cnt = z2h.z2h_circuit_step(Lx, Ly, cx, cz, dt, 0)
    g = z2h.gates_to_list(arr, cnt)
    assert cnt == 3 * n + 52 * nv
    if (Lx, Ly) == (3, 3):
        assert cnt == 522
    assert [k for k, *_ in g[:n]] == [z2h.Z2H_GATE_RX] * n
    assert all(abs(t - (-cx[2] * dt)) < 1e-15 for _, _, _, t in g[:n])
    assert all(q1 == n for k, q0, q1, _ in g if k == z2h.Z2H_GATE_CNOT)
    anc_rz = [t for k, q0, _, t in g if k == z2h.Z2H_GATE_RZ and q0 == n]
    assert sorted(set(round(t, 15) for t in anc_rz)) == sorted({round(-cz[1] * dt, 15), round(-cx[0] * dt, 15)})
    assert len(anc_rz) == 2 * 2 * nv
    link_rz = [t for k, q0, _, t in g if k == z2h.Z2H_GATE_RZ and q0 < n]
    assert len(link_rz) == n and all(abs(t + 2 * cz[3] * dt) < 1e-15 for t in link_rz)
    st, pl = z2h.z2h_masks(Lx, Ly)
    # the first gadget belongs to plaquette 0: CNOTs from exactly its links
    first = g[n:n + 4]
    assert sum(1 << q0 for _, q0, _, _ in first) == int(pl[0])


def test_circuit_prep_structure():
    arr, cnt = z2h.z2h_circuit_prep(3, 3, z2h.Z2H_INIT_PSI1)
    g = z2h.gates_to_list(arr, cnt)
    assert cnt == 18 + 9 * 9 + 1
    assert g[-1][0] == z2h.Z2H_GATE_NORM
    assert sum(1 for k, *_ in g if k == z2h.Z2H_GATE_PROJ0) == 9
    arr, cnt = z2h.z2h_circuit_prep(3, 3, z2h.Z2H_INIT_PSI1P)
    assert cnt == 9 * (4 + 4 + 1 + 4 + 4) + 1
    with pytest.raises(z2h.Z2HError):
        z2h.z2h_circuit_prep(3, 3, z2h.Z2H_INIT_PLUS)


def test_gate_list_validation():
    """Rejections that happen before any device work."""
    G = z2h.z2h_gate
    ws = np.zeros(4096, np.uint8)

    def run(nq, gates, fuse=0):
        arr = (G * len(gates))(*[G(*g) for g in gates])
        code = z2h.lib().z2h_gates_run(nq, z2h.Z2H_C128, ctypes.c_void_p(256), ws.ctypes.data_as(ctypes.c_void_p),
                                       ws.nbytes, arr, len(gates), fuse, None)
        return code

    assert run(5, [(z2h.Z2H_GATE_H, 5, 0, 0, 0.0)]) == -1          # qubit out of range
    assert run(5, [(z2h.Z2H_GATE_CNOT, 1, 1, 0, 0.0)]) == -1       # control == target
    assert run(5, [(9, 0, 0, 0, 0.0)]) == -1                       # unknown kind
    assert run(1, [(z2h.Z2H_GATE_H, 0, 0, 0, 0.0)]) == -1          # nq too small
    assert run(35, [(z2h.Z2H_GATE_H, 0, 0, 0, 0.0)]) == -1         # nq too large
    assert run(5, [(z2h.Z2H_GATE_RX, 0, 0, 0, float("nan"))]) == -1
    assert z2h.z2h_gates_ws_bytes(1) == 0 and z2h.z2h_gates_ws_bytes(19) >= 8 * 2048
    cnt = ctypes.c_int32()
    code = z2h.lib().z2h_circuit_step(3, 3, ctypes.byref(z2h.couplings()), ctypes.byref(z2h.couplings()), 0.1, 0,
                                      None, 0, ctypes.byref(cnt))
    assert code == -6 and cnt.value == 522


def test_exact_solver_workspace_checks():
    """Lanczos and the Krylov evolution reject a workspace below the stated
    size, and overlapping buffers, before any device work."""
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    L = z2h.lib()
    need = z2h.z2h_lanczos_sizes(plan, 40)
    it, e0 = ctypes.c_int32(), ctypes.c_double()
    H = z2h.couplings(0.5, 0.5, 0.2, 0.1)
    v, ws = ctypes.c_void_p(1 << 40), ctypes.c_void_p((1 << 40) + (1 << 30))
    code = L.z2h_lanczos_ground(plan.handle, v, ws, need - 256, ctypes.byref(H), 40, 1e-10, None, None,
                                ctypes.byref(it), ctypes.byref(e0), None)
    assert code == -6
    code = L.z2h_lanczos_ground(plan.handle, v, ctypes.c_void_p((1 << 40) + 4096), need, ctypes.byref(H), 40, 1e-10,
                                None, None, ctypes.byref(it), ctypes.byref(e0), None)
    assert code == -1 and b"overlap" in L.z2h_last_error()
    sched = z2h.schedule((0.5, 0.5, 0, 0), (0.5, 0.5, 0.3, 0.2), 10, 0.1)
    err = ctypes.c_double()
    need = z2h.z2h_exact_sizes(plan, 12)
    code = L.z2h_exact_evolve(plan.handle, v, ws, need - 256, ctypes.byref(sched), 12, ctypes.byref(err), None)
    assert code == -6
    code = L.z2h_hamiltonian_apply(plan.handle, v, ctypes.c_void_p((1 << 40) + 256), ctypes.byref(H), None)
    assert code == -1 and b"overlap" in L.z2h_last_error()


def _gate_array(lib_gates):
    arr = (z2h.z2h_gate * max(len(lib_gates), 1))()
    for a, (k, q0, q1, th) in zip(arr, lib_gates):
        a.kind, a.q0, a.q1, a.theta = k, q0, q1, th
    return arr


def test_gate_schedule_pass_counts():
    """Commutation-aware grouping of the 4x4 Trotter-step circuit (928 gates,
    33 qubits): 32 tile passes in complex64 (tile of 13 qubits), 33 in
    complex128 (12), 71 register passes (five qubits; one per gadget, 64, is
    the floor), every gate its own pass gate by gate."""
    arr, ng = z2h.z2h_circuit_step(4, 4, (0.5, 0.5, 0.3, 0.2), (0.5, 0.5, 0.3, 0.2), 0.1)
    assert ng == 928
    assert z2h.z2h_gates_schedule(33, z2h.Z2H_C64, arr, ng, 1)[1] == 32
    assert z2h.z2h_gates_schedule(33, z2h.Z2H_C128, arr, ng, 1)[1] == 33
    assert z2h.z2h_gates_schedule(33, z2h.Z2H_C64, arr, ng, 2)[1] == 71
    assert z2h.z2h_gates_schedule(33, z2h.Z2H_C64, arr, ng, 0) == (list(range(928)), 928)


@pytest.mark.parametrize("nq,fuse,dtype", [(12, 1, 0), (12, 2, 0), (15, 1, 1), (16, 2, 1), (8, 2, 0), (5, 1, 0)])
def test_gate_schedule_is_a_valid_reordering(nq, fuse, dtype):
    """Random gate lists with renormalisations: a gate never passes an
    earlier gate on one of its qubits, renormalisations are passes of their
    own that nothing crosses, each pass fits the executor's qubit limit, and
    applying the gates in executed order (pass, then index) gives the state
    of the written order (oracle circuit application)."""
    from oracle import circuit
    rng = np.random.default_rng(77 + nq + 10 * fuse)
    tile = min(nq, {0: 13, 1: 12}[dtype])
    K = 5 if (fuse == 2 and nq >= 11) else tile
    base = 0xF if (fuse == 1 or nq < 11) else 0
    lib, ora = [], []
    for i in range(160):
        r = rng.random()
        if i in (50, 51, 120):
            lib.append((z2h.Z2H_GATE_NORM, 0, 0, 0.0))
            ora.append(("NORM", ()))
        elif r < 0.4:
            c, t = (int(x) for x in rng.choice(nq, 2, replace=False))
            lib.append((z2h.Z2H_GATE_CNOT, c, t, 0.0))
            ora.append(("CNOT", (c, t)))
        else:
            q, th = int(rng.integers(nq)), float(rng.uniform(-2, 2))
            k = ("H", "RX", "RZ")[int(rng.integers(3))]
            lib.append(({"H": z2h.Z2H_GATE_H, "RX": z2h.Z2H_GATE_RX, "RZ": z2h.Z2H_GATE_RZ}[k], q, 0, th))
            ora.append((k, (q,)) if k == "H" else (k, (q,), th))
    pass_of, npasses = z2h.z2h_gates_schedule(nq, dtype, _gate_array(lib), len(lib), fuse)
    assert sorted(set(pass_of)) == list(range(npasses))
    if nq < 6:
        assert pass_of == list(range(len(lib)))
        return

    def qubits(g):
        k, q0, q1, _ = g
        return {q0, q1} if k == z2h.Z2H_GATE_CNOT else {q0}
    for i, gi in enumerate(lib):
        for j in range(i + 1, len(lib)):
            gj = lib[j]
            if gi[0] == z2h.Z2H_GATE_NORM or gj[0] == z2h.Z2H_GATE_NORM:
                assert pass_of[i] < pass_of[j]
            elif qubits(gi) & qubits(gj):
                assert pass_of[i] <= pass_of[j]
    for p in range(npasses):
        members = [lib[i] for i in range(len(lib)) if pass_of[i] == p]
        if members[0][0] == z2h.Z2H_GATE_NORM:
            assert len(members) == 1
            continue
        used = base
        for g in members:
            for q in qubits(g):
                used |= 1 << q
        assert bin(used).count("1") <= K
    order = sorted(range(len(lib)), key=lambda i: (pass_of[i], i))
    x = rng.normal(size=1 << nq) + 1j * rng.normal(size=1 << nq)
    a = circuit.apply(x, ora)
    b = circuit.apply(x, [ora[i] for i in order])
    assert np.abs(a - b).max() < 1e-12


def test_gate_schedule_validation():
    """z2h_gates_schedule rejects what z2h_gates_run rejects, and NULL
    outputs; a valid call writes one pass index per gate."""
    G = z2h.z2h_gate
    L = z2h.lib()
    out = (ctypes.c_int32 * 4)()
    npass = ctypes.c_int32()

    def sched(nq, gates, fuse=1, dtype=z2h.Z2H_C64, pass_of=out, np_=ctypes.byref(npass)):
        arr = (G * max(len(gates), 1))(*[G(*g) for g in gates])
        return L.z2h_gates_schedule(nq, dtype, arr, len(gates), fuse, pass_of, np_)

    h0 = (z2h.Z2H_GATE_H, 0, 0, 0, 0.0)
    assert sched(12, [(z2h.Z2H_GATE_H, 12, 0, 0, 0.0)]) == -1     # qubit out of range
    assert sched(12, [(z2h.Z2H_GATE_CNOT, 3, 3, 0, 0.0)]) == -1   # control == target
    assert sched(12, [h0], fuse=3) == -1                            # unknown executor
    assert sched(12, [h0], dtype=7) == -1                           # unknown dtype
    assert sched(1, [h0]) == -1 and sched(35, [h0]) == -1            # nq out of range
    assert sched(12, [h0], pass_of=None) == -1                      # NULL output
    assert sched(12, [h0], np_=None) == -1
    assert sched(12, []) == 0 and npass.value == 0                   # empty list
    gates = [h0, (z2h.Z2H_GATE_CNOT, 0, 11, 0, 0.0), (z2h.Z2H_GATE_NORM, 0, 0, 0, 0.0), (z2h.Z2H_GATE_RZ, 5, 0, 0, 0.3)]
    assert sched(12, gates) == 0 and npass.value == 3 and list(out) == [0, 0, 1, 2]
    assert sched(12, gates, fuse=0) == 0 and npass.value == 4 and list(out) == [0, 1, 2, 3]


def test_binding_covers_the_header():
    """Every function declared in include/z2h.h has a ctypes signature and a
    wrapper of the same name in the Python binding."""
    hdr = open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "include", "z2h.h")).read()
    names = set(re.findall(r"^\s*(?:z2h_status|size_t|int32_t|const char \*|void|double|uint64_t)\s+\**(z2h_[a-z0-9_]+)\s*\(",
                           hdr, re.M))
    assert len(names) > 40
    src = open(z2h.__file__).read()
    assert not [n for n in names if f'"{n}"' not in src]
    assert not [n for n in names if not callable(getattr(z2h, n, None))]


def test_size_queries_through_the_binding():
    """The two size queries other wrappers use internally, called directly."""
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    assert z2h.z2h_lanczos_vector_sizes(plan, 40) > 0
    p = z2h.make_path([(1, 1, 0, 0), (1, 1, 0.3, 0.3)], [100], 0.02, every=10)
    samples, ws = z2h.z2h_paths_sizes(plan, [p, p])
    assert samples == 11 and ws > 0
