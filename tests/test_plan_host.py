"""The host-side sphere -> box map builder (csrc/plan_host.cpp), built with
g++ and AddressSanitizer + UndefinedBehaviorSanitizer and run on the CPU:
every array it hands to the FFT kernels is checked against its definition
(columns = points of equal (m1, m2) along N3, ordered by centred m1, m2, m3;
extent = distinct m1), on spheres of the benchmark's kind, reordered and
holed spheres, wrapped Miller indices, degenerate boxes and a box too small
for its sphere."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_08578_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("plan") / "plan_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(CSRC, "plan_host.cpp"),
           os.path.join(ROOT, "tests", "plan_driver.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def run(driver, box, miller):
    miller = np.asarray(miller, dtype=np.int64).reshape(-1, 3)
    text = f"{box[0]} {box[1]} {box[2]} {len(miller)}\n" + "\n".join(
        " ".join(str(int(v)) for v in row) for row in miller) + "\n"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1")
    res = subprocess.run([driver], input=text, capture_output=True, text=True, env=env,
                         timeout=120)
    assert res.returncode == 0, res.stderr[-2000:]
    out = {}
    for line in res.stdout.splitlines():
        k, *v = line.split()
        out[k] = np.array([int(x) for x in v], dtype=np.int64)
    return out


def centred(m, n):
    return np.where(m <= n // 2, m, m - n)


def check_plan(out, box, miller):
    n1, n2, n3 = box
    miller = np.asarray(miller, dtype=np.int64).reshape(-1, 3)
    npw = len(miller)
    assert out["rc"][0] == 0
    ncols, ldt, xr, quarter12, runs = (int(x) for x in out["scalars"])
    m = np.stack([miller[:, 0] % n1, miller[:, 1] % n2, miller[:, 2] % n3], axis=1)
    c = np.stack([centred(m[:, 0], n1), centred(m[:, 1], n2), centred(m[:, 2], n3)], axis=1)
    perm = out["pt_perm"]
    assert sorted(perm.tolist()) == list(range(npw))
    # column order: lexicographic in centred (m1, m2, m3), stable for ties (none: cells distinct)
    key = c[perm]
    assert all(tuple(key[i]) < tuple(key[i + 1]) for i in range(npw - 1))
    cols = sorted(set(map(tuple, c[:, :2].tolist())))
    assert ncols == len(cols) and ldt % 16 == 0 and ncols <= ldt < ncols + 16
    cs = out["col_start"]
    assert len(cs) == ncols + 1 and cs[0] == 0 and cs[-1] == npw and np.all(np.diff(cs) > 0)
    ext = sorted(set(c[:, 0].tolist()))
    assert xr == len(ext)
    assert np.array_equal(centred(out["ext_m1"], n1), np.array(ext))
    for j, (a1, a2) in enumerate(cols):
        pts = perm[cs[j]:cs[j + 1]]
        assert np.all(c[pts, 0] == a1) and np.all(c[pts, 1] == a2)
        assert np.all(out["pt_col"][cs[j]:cs[j + 1]] == j)
        assert out["col_m2"][j] == a2 % n2
        assert out["ext_m1"][out["col_e"][j]] == a1 % n1
        assert out["col_m3lo"][j] == c[pts[0], 2]
    assert np.array_equal(out["pt_m3"], m[perm, 2])
    want_runs = int(np.array_equal(perm, np.arange(npw)) and all(
        np.all(np.diff(c[perm[cs[j]:cs[j + 1]], 2]) == 1) for j in range(ncols)))
    assert runs == want_runs
    want_q = int(np.all(4 * c[:, 0] >= -n1) and np.all(4 * c[:, 0] < n1) and
                 np.all(4 * c[:, 1] >= -n2) and np.all(4 * c[:, 1] < n2))
    assert quarter12 == want_q
    return runs, quarter12


def sphere(name):
    if name == "c1":
        w = synth.config_c1()
    else:
        w = synth.config_c4(ncells=8)[3]
    return list(w.box), np.asarray(w.miller, dtype=np.int64)


@pytest.mark.parametrize("name", ["c1", "c4_cell3"])
def test_sphere_in_column_order(driver, name):
    box, miller = sphere(name)
    runs, q = check_plan(run(driver, box, miller), box, miller)
    assert runs == 1


def test_shuffled_and_holed_spheres(driver):
    box, miller = sphere("c1")
    rng = np.random.default_rng(0)
    shuffled = miller[rng.permutation(len(miller))]
    assert check_plan(run(driver, box, shuffled), box, shuffled)[0] == 0
    # drop a point from the middle of the longest column: a gap along N3
    key = [tuple(r) for r in miller[:, :2].tolist()]
    longest = max(set(key), key=key.count)
    idx = [i for i, k in enumerate(key) if k == longest]
    holed = np.delete(miller, idx[len(idx) // 2], axis=0)
    assert check_plan(run(driver, box, holed), box, holed)[0] == 0


def test_wrapped_indices_and_degenerate_boxes(driver):
    rng = np.random.default_rng(1)
    box = (12, 10, 9)
    cells = rng.choice(12 * 10 * 9, size=200, replace=False)
    m = np.stack([cells % 12, (cells // 12) % 10, cells // 120], axis=1)
    wrapped = m + np.array([12, -10, 9]) * rng.integers(-3, 4, size=(200, 3))
    check_plan(run(driver, box, wrapped), box, wrapped)
    check_plan(run(driver, (1, 1, 1), [[5, -7, 2]]), (1, 1, 1), [[5, -7, 2]])
    line = [[0, 0, k] for k in range(-3, 4)]
    assert check_plan(run(driver, (1, 1, 7), line), (1, 1, 7), line) == (1, 1)


def test_box_too_small_names_the_point(driver):
    box, miller = sphere("c1")
    small = (box[0] // 2, box[1], box[2])
    out = run(driver, small, miller)
    assert out["rc"][0] == 1
    bad = int(out["bad"][0])
    m = np.stack([miller[:, 0] % small[0], miller[:, 1] % small[1], miller[:, 2] % small[2]], 1)
    seen = {tuple(r) for r in m[:bad].tolist()}
    assert len(seen) == bad and tuple(m[bad]) in seen


def test_arguments_out_of_range(driver):
    assert run(driver, (0, 4, 4), [[0, 0, 0]])["rc"][0] == 2
    assert run(driver, (4, 4, 5000), [[0, 0, 0]])["rc"][0] == 2
