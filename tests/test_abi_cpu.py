"""C ABI checks that need no GPU: the library loads and exports every entry
point include/snake.h declares, the ctypes descriptor matches the C layout,
and descriptor validation rejects bad input before touching the device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1904_02833_amd as snk
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "snake.h")
MLP_HEADER = os.path.join(ROOT, "include", "snake_mlp.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(snk.LIB_PATH):
        from paper_1904_02833_amd import build
        build.build()
    return snk.lib()


def declared_functions(path=HEADER, prefix="sim_"):
    text = open(path).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|void|const char\*)\s+(" + prefix + r"\w+)\s*\(",
                                 text, re.M)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert set(names) == set(snk.EXPORTS)
    mlp_names = declared_functions(MLP_HEADER, "mlp_")
    assert set(mlp_names) == set(snk.MLP_EXPORTS)
    names = names + mlp_names
    out = subprocess.run(["nm", "-D", "--defined-only", snk.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T ((?:sim|mlp)_\w+)$", out, re.M))
    for n in names:
        assert n in exported, n
        assert hasattr(L, n)


def test_state_fields_match_the_header():
    """The binding's field table names the header's SIM_F_* bits in order,
    with SIM_F_COUNT entries."""
    text = open(os.path.join(ROOT, "include", "snake.h")).read()
    bits = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define SIM_F_(\w+) \(1u << (\d+)\)", text)}
    count = int(re.search(r"#define SIM_F_COUNT (\d+)", text).group(1))
    assert len(snk.FIELDS) == count == len(bits)
    for k, f in enumerate(snk.FIELDS):
        assert bits[f[0].upper()] == k, f[0]


def test_descriptor_layout_matches_c(tmp_path):
    """Compile a probe against the header with gcc and compare sizeof and
    every field offset with the ctypes mirror."""
    fields = [f[0] for f in snk.Desc._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "snake.h"', 'int main(void){',
           'printf("%zu\\n", sizeof(sim_desc_t));']
    src += [f'printf("%zu\\n", offsetof(sim_desc_t, {f}));' for f in fields]
    src += ["return 0;}"]
    c = tmp_path / "probe.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0] == C.sizeof(snk.Desc)
    for f, off in zip(fields, vals[1:]):
        assert getattr(snk.Desc, f).offset == off, f


def test_oracle_batch_layout_matches_c(tmp_path):
    import oracle
    fields = [f[0] for f in oracle.Batch._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "snake_oracle.h"',
           'int main(void){', 'printf("%zu\\n", sizeof(orc_batch));']
    src += [f'printf("%zu\\n", offsetof(orc_batch, {f}));' for f in fields]
    src += ["return 0;}"]
    c = tmp_path / "probe.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "oracle"), str(c), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0] == C.sizeof(oracle.Batch)
    for f, off in zip(fields, vals[1:]):
        assert getattr(oracle.Batch, f).offset == off, f


def ws_bytes(L, wl, **over):
    d, keep = snk.make_desc(wl, **over)
    n = C.c_size_t(0)
    rc = L.sim_workspace_bytes(C.byref(d), C.byref(n))
    return rc, n.value, L.sim_last_error().decode()


def test_workspace_bytes_valid_and_monotone(L):
    rc1, b1, _ = ws_bytes(L, W.make("uniform", n_snakes=16))
    rc2, b2, _ = ws_bytes(L, W.make("uniform", n_snakes=64))
    assert rc1 == rc2 == 0
    assert 0 < b1 < b2
    rc, b, _ = ws_bytes(L, W.make("uneven", n_snakes=50).take(
        np.nonzero((W.make("uneven", n_snakes=50).bodies) <= 64)[0]))
    assert rc == 0 and b > 0


@pytest.mark.parametrize("field,value,msg", [
    ("n_modules", np.zeros(2, np.int32), "n_modules"),
    ("alpha_bend", np.array([1e-5, np.nan]), "compliance"),
    ("mu", np.array([0.5, -1.0]), "mu"),
    ("dt", 0.0, "dt"),
    ("substeps", 0, "substeps"),
    ("iters", -1, "iters"),
    ("relax", 1.5, "relax"),
    ("tau_inflate", 0.0, "tau"),
    ("controller", 7, "controller"),
    ("flags", 64, "flag"),
    ("map_rows", 3, "map_rows"),
    ("mlp_fallback_k", 21, "mlp_fallback_k"),
    ("mlp_fallback_k", -1, "mlp_fallback_k"),
])
def test_descriptor_validation(L, field, value, msg):
    wl = W.custom([2, 2], 8)
    rc, _, err = ws_bytes(L, wl, **{field: value})
    assert rc == snk.SIM_EINVAL
    assert msg in err


@pytest.mark.parametrize("over,msg", [
    (dict(solver=3), "solver"),
    (dict(solver=1, warm_start=2), "zero or the previous"),
    (dict(solver=2, warm_start=1), "zero multipliers"),
    (dict(solver=1, newton_iters=-1), "newton_iters"),
    (dict(solver=1, newton_iters=10001), "newton_iters"),
    (dict(solver=1, pcr_iters=0), "pcr_iters"),
    (dict(solver=1, newton_keep_best=2), "newton_keep_best"),
    (dict(flags=16, solver=1), "wheel carriage"),
    (dict(flags=16, solver=2), "wheel carriage"),
    (dict(flags=16, warm_start=1), "wheel carriage"),
    (dict(flags=16, warm_start=2), "wheel carriage"),
])
def test_solver_descriptor_validation(L, over, msg):
    rc, _, err = ws_bytes(L, W.custom([2, 2], 8), **over)
    assert rc == snk.SIM_EINVAL
    assert msg in err


def test_newton_workspace_adds_its_arrays(L):
    wl = W.make("uneven", n_snakes=40)
    rc0, b0, _ = ws_bytes(L, wl)
    rc1, b1, _ = ws_bytes(L, wl, solver=1, newton_iters=4, pcr_iters=20)
    assert rc0 == rc1 == 0 and b1 > b0


def test_carriage_workspace_adds_the_wheels(L):
    """Wheel state (segments x 2 wheels x 22 floats) and the lane-class list
    and double compliances of the carriage kernel."""
    wl = W.make("uneven", n_snakes=40)
    rc0, b0, _ = ws_bytes(L, wl)
    rc1, b1, _ = ws_bytes(L, wl, flags=16)
    assert rc0 == rc1 == 0
    assert b1 - b0 >= 2 * 22 * 4 * int(wl.bodies.sum())


def test_schedule_validation(L):
    wl = W.custom([1, 1], 8, controller=W.CTRL_SCHEDULE)
    wl.sched_off = np.array([0, 1, 1], np.int32)     # second module has no piece
    wl.sched_steps = np.array([5], np.int32)
    wl.sched_val = np.array([0.5])
    rc, _, err = ws_bytes(L, wl)
    assert rc == snk.SIM_EINVAL and "piece" in err


def test_create_rejects_bad_workspace_without_device(L):
    wl = W.custom([2], 8)
    d, keep = snk.make_desc(wl)
    h = C.c_void_p()
    assert L.sim_create(C.byref(d), None, 1 << 20, None, C.byref(h)) == snk.SIM_EINVAL
    assert L.sim_create(C.byref(d), C.c_void_p(4096 + 8), 1 << 20, None, C.byref(h)) == snk.SIM_EINVAL
    assert L.sim_create(C.byref(d), C.c_void_p(4096), 16, None, C.byref(h)) == snk.SIM_ENOMEM
    assert "workspace too small" in L.sim_last_error().decode()
    assert not h.value


def test_null_handles(L):
    L.sim_destroy(None)
    assert L.sim_step(None, 1) == snk.SIM_EINVAL
    assert L.sim_set_pressures(None, None, 0, 0) == snk.SIM_EINVAL
    assert L.sim_read_state(None, 1, None, 0) == snk.SIM_EINVAL
    assert L.sim_read_index(None, 0, None, 0) == snk.SIM_EINVAL


def check_plan(wl, waves, min_seg, rows):
    hdr, slots = snk.plan_tiles(wl, waves, min_seg, rows)
    B = np.asarray(wl.n_modules, np.int64) * np.asarray(wl.segs_per_module, np.int64)
    cap = 64 * waves
    seen = np.zeros(len(B), np.int64)
    prev_first = None
    for t, (first, count, crosses, rw) in enumerate(hdr):
        assert count >= 1 and rw == rows
        used = np.zeros(cap, bool)
        cross = False
        for k in range(first, first + count):
            s, code = slots[k]
            off, seg = int(code) >> 16, int(code) & 0xFFFF
            seen[s] += 1
            assert seg >= B[s] and off + seg <= cap
            if rows == 2 and B[s] <= 8:
                assert seg == 8 and off % 8 == 0
            elif rows:
                assert off % 16 == 0 and seg == (B[s] + 15) // 16 * 16
            else:
                assert seg == max(min_seg, 1 << int(np.ceil(np.log2(B[s])))) and off % seg == 0
            assert not used[off:off + seg].any()
            used[off:off + seg] = True
            cross |= (off // 64) != ((off + seg - 1) // 64)
        assert bool(crosses) == cross
        # tiles in work order: the snake that opened a tile is no shorter than the next tile's
        b0 = B[slots[first][0]]
        if prev_first is not None:
            assert b0 <= prev_first
        prev_first = b0
    assert np.all(seen == 1)
    return hdr, slots, B


@pytest.mark.parametrize("waves,min_seg,rows", [(4, 16, 0), (4, 32, 0), (8, 64, 0), (4, 16, 1), (16, 16, 1)])
def test_tile_plan_places_every_snake_once(L, waves, min_seg, rows):
    """Host tile packing: every snake once, segments inside their tile and
    disjoint, sizes and alignment of the layout, wave-crossing flags."""
    wl = W.make("uneven", n_snakes=3000)
    check_plan(wl, waves, min_seg, rows)


def test_tile_plan_half_rows_pair_short_snakes(L):
    """Half rows: snakes of up to 8 bodies take 8 lanes, two consecutive
    ones (in work order) sharing a 16-lane row; a mixed batch keeps the
    longer snakes' segments on whole rows.  The short batch (6 to 8 bodies)
    then fills at least 75 % of its lanes, against under half with whole
    rows."""
    wl = W.make("short", n_snakes=1000)
    hdr2, slots2, B = check_plan(wl, 4, 16, 2)
    hdr1, _, _ = check_plan(wl, 4, 16, 1)
    fill2 = B.sum() / (len(hdr2) * 256)
    fill1 = B.sum() / (len(hdr1) * 256)
    print(f"half rows {fill2:.3f}, whole rows {fill1:.3f}")
    assert fill2 >= 0.75 and fill1 < 0.5
    mixed = W.custom([1] * 9, [3, 17, 8, 5, 1, 40, 2, 9, 7])
    check_plan(mixed, 1, 16, 2)
    check_plan(mixed, 2, 16, 2)


def test_tile_plan_rows_layout_fills_lanes(L):
    """Best-fit rows layout of the uneven batch keeps at least 90 % of the
    lanes busy; the aligned layout of the same batch stays near 72 %."""
    wl = W.make("uneven", n_snakes=4000)
    hdr_r, _, B = check_plan(wl, 4, 16, 1)
    hdr_a, _, _ = check_plan(wl, 4, 16, 0)
    fill_r = B.sum() / (len(hdr_r) * 256)
    fill_a = B.sum() / (len(hdr_a) * 256)
    print(f"\n[plan] lanes busy: rows {fill_r:.3f} aligned {fill_a:.3f}")
    assert fill_r >= 0.90 and fill_a < 0.8


def test_tile_plan_rejects_bad_mapping(L):
    wl = W.make("uneven", n_snakes=50)
    for args in [(3, 16, 0), (4, 8, 0), (4, 16, 3), (4, 16, -1), (1, 16, 0)]:
        with pytest.raises(snk.SimError):
            snk.plan_tiles(wl, *args)


def test_empty_and_oversized_batches_rejected(L):
    wl = W.custom([2], 8)
    rc, _, err = ws_bytes(L, wl, n_modules=np.zeros(0, np.int32), segs_per_module=np.zeros(0, np.int32))
    assert rc == snk.SIM_EINVAL
    big = W.custom([9], 128)             # 1152 bodies
    rc, _, err = ws_bytes(L, big)
    assert rc == snk.SIM_EINVAL and "1024" in err
    edge = W.custom([8], 128)            # exactly 1024 bodies
    rc, b, _ = ws_bytes(L, edge)
    assert rc == 0 and b > 0


def test_wheel_batch_size_limit(L):
    """The carriage indexes its wheel multipliers (9 components of 2N wheels)
    with 32-bit offsets, so a wheel batch stops below 2^31 / 18 bodies; the
    same batch without wheels is accepted (its limit is 2^28)."""
    limit = (1 << 31) // 18 - 1
    n = limit // 1024 + 1                      # snakes of 1024 bodies
    big = W.custom(np.full(n, 8, np.int32), 128)
    assert int(big.bodies.sum()) > limit
    rc, _, err = ws_bytes(L, big, flags=16)
    assert rc == snk.SIM_EINVAL and "wheel carriage" in err
    rc, b, _ = ws_bytes(L, big)
    assert rc == 0 and b > 0
    ok = W.custom(np.full(n - 1, 8, np.int32), 128)
    assert int(ok.bodies.sum()) <= limit
    rc, b, _ = ws_bytes(L, ok, flags=16)
    assert rc == 0 and b > 0


# ---------------------------------------------------------------- full-resolution link (include/link.h)

LINK_HEADER = os.path.join(ROOT, "include", "link.h")


def test_link_exports_every_declared_symbol(L):
    from paper_1904_02833_amd import link as LK

    names = declared_functions(LINK_HEADER, "link_")
    assert set(names) == set(LK.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", snk.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (link_\w+)$", out, re.M))
    for n in names:
        assert n in exported, n
        assert hasattr(LK.lib(), n)


def test_link_fields_and_index_match_the_header():
    from paper_1904_02833_amd import link as LK

    text = open(LINK_HEADER).read()
    bits = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define LINK_F_(\w+) \(1u << (\d+)\)", text)}
    count = int(re.search(r"#define LINK_F_COUNT (\d+)", text).group(1))
    assert len(LK.FIELDS) == count == len(bits)
    for k, f in enumerate(LK.FIELDS):
        assert bits[f[0].upper()] == k, f[0]
    idx = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define LINK_IDX_(\w+) (\d+)", text)}
    names = {"DIST_I": "dist_i", "DIST_J": "dist_j", "DIST_KIND": "dist_kind", "DEG_PARTICLE": "degree_particle",
             "DEG_FRAME": "degree_frame"}
    for key, name in names.items():
        assert LK.INDEX.index(name) == idx[key]


def test_link_descriptor_layout_matches_c(tmp_path):
    from paper_1904_02833_amd import link as LK

    fields = [f[0] for f in LK.LinkDesc._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "link.h"', 'int main(void){',
           'printf("%zu\\n", sizeof(link_desc_t));']
    src += [f'printf("%zu\\n", offsetof(link_desc_t, {f}));' for f in fields]
    src += ["return 0;}"]
    c = tmp_path / "probe.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals[0] == C.sizeof(LK.LinkDesc)
    for f, off in zip(fields, vals[1:]):
        assert getattr(LK.LinkDesc, f).offset == off, f


def test_link_validation_and_workspace(L):
    """Descriptor checks run on the host: sizes grow with the batch, bad
    input is refused with a message, nothing touches a device."""
    from paper_1904_02833_amd import link as LK

    wl = W.make_link(4, n_links=4)
    b4 = LK.workspace_bytes(wl)
    b8 = LK.workspace_bytes(W.make_link(8, n_links=4))
    assert b8 > b4 > 0
    for over, msg in ((dict(n_links=5), "n_links"), (dict(ring=6), "ring"), (dict(poisson=0.5), "material"),
                      (dict(relax=0.0), "relax"), (dict(iters=-1), "iters"), (dict(flags=64), "flag"),
                      (dict(rigid_compliance=-1.0), "rigid_compliance"), (dict(sections=2), "sections")):
        with pytest.raises(LK.LinkError) as e:
            LK.workspace_bytes(wl, **over)
        assert e.value.code == -1 and msg in str(e.value), (over, str(e.value))
    bad = wl.tets.copy()
    bad[3, 2] = 999
    with pytest.raises(LK.LinkError):
        LK.workspace_bytes(wl, tets=bad)
    big = W.make_link(1, n_links=4, sections=30)
    with pytest.raises(LK.LinkError):
        LK.workspace_bytes(big)


def _link_incidence_counts(sections, ring, tets):
    """Blocks touching each particle of a link, counted from the mesh: its
    tetrahedra, the axial rows to the same slot of the neighbouring
    sections, the radial rows between an inner section's centre and its
    ring, and the end sections' attachments."""
    n = ring + 1
    cnt = np.bincount(np.asarray(tets).ravel(), minlength=sections * n).astype(np.int64)
    for g in range(sections):
        for s in range(n):
            p = g * n + s
            cnt[p] += (g > 0) + (g < sections - 1)
            if 0 < g < sections - 1:
                cnt[p] += ring if s == 0 else 1
            if g == 0 or g == sections - 1:
                cnt[p] += 1
    return cnt


@pytest.mark.parametrize("sections,ring,n_links", [(13, 8, 4), (5, 4, 4), (7, 12, 2), (13, 8, 1)])
def test_link_gather_plan_covers_every_incidence_entry_once(L, sections, ring, n_links):
    """The kernel's lane plan (host only): every particle owns one aligned
    group of 1-8 lanes within a wave, below the frames' wave; the group's
    ranges follow one another and cover the particle's incidence list
    exactly, the lists of a link particle by particle, each range within
    the group's even share."""
    from paper_1904_02833_amd import link as LK

    wl = W.make_link(1, n_links=n_links, sections=sections, ring=ring)
    part, size, first, end, gmax = LK.plan_gathers(wl)
    P1 = sections * (ring + 1)
    cnt = _link_incidence_counts(sections, ring, wl.tets)
    off = np.concatenate([[0], np.cumsum(cnt)])
    n_inc = 4 * len(wl.tets) + 2 * ((sections - 1) * (ring + 1) + (sections - 2) * ring) + 2 * (ring + 1)
    assert off[-1] == n_inc
    assert np.all(part[960:] == -1)
    assert gmax == size.max() and gmax in (1, 2, 4, 8)
    for p in range(n_links * P1):
        lanes = np.flatnonzero(part == p)
        g = len(lanes)
        assert g >= 1 and np.all(size[lanes] == g), p
        assert lanes[0] % g == 0 and np.array_equal(lanes, lanes[0] + np.arange(g)), p
        pk = p % P1
        assert first[lanes[0]] == off[pk] and end[lanes[-1]] == off[pk + 1], p
        assert np.array_equal(first[lanes[1:]], end[lanes[:-1]]), p
        assert np.all(end[lanes] - first[lanes] <= -(-cnt[pk] // g)), p
    assert np.sum(part >= 0) == np.sum(size[part >= 0] > 0)
