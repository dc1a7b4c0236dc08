"""The host half of the library (model validation, the path and pair tables,
feature segments, output groups, the Gauss-Legendre rule) compiled with g++
under AddressSanitizer and UndefinedBehaviorSanitizer and run on valid,
multi-output, wide and malformed models.  Any sanitizer report fails the
test; the tables' sizes must equal the library's own host-only build."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2605_04497_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("san") / "host_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(HERE, "sanitize", "host_driver.cpp"),
           os.path.join(CSRC, "host", "path_table.cpp"),
           os.path.join(CSRC, "host", "dfs_table.cpp"),
           os.path.join(CSRC, "host", "gauss_legendre.cpp"), "-o", out]
    subprocess.check_call(cmd)
    return out


def _write(path, ens):
    T, N = ens.n_trees, ens.n_nodes
    K = int(getattr(ens, "n_groups", 1) or 1)
    tg = ens.tree_group if ens.tree_group is not None else np.zeros(T, np.int32)
    base = np.broadcast_to(np.asarray(ens.base_score, np.float64).reshape(-1), (K,))
    with open(path, "wb") as f:
        f.write(np.array([T, ens.n_features, K, N], np.int32).tobytes())
        f.write(np.asarray(ens.tree_offsets, np.int64).tobytes())
        for a, dt in ((ens.left, np.int32), (ens.right, np.int32), (ens.feature, np.int32),
                      (ens.threshold, np.float32), (ens.default_left, np.uint8),
                      (ens.cover, np.float64), (ens.value, np.float64),
                      (tg, np.int32), (base, np.float64)):
            f.write(np.ascontiguousarray(a, dt).tobytes())


def _run(driver, tmp_path, ens):
    p = str(tmp_path / "model.bin")
    _write(p, ens)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, p], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, \
        r.stderr[-4000:]
    return r.stdout.strip()


MODELS = [
    ("c1_small", dict(M=4)),
    ("c3_interactions", dict(T=5, M=4, n_train=20000)),
    ("c5_deep", dict(T=3, M=4, n_train=30000)),
    ("c2_values", dict(T=6, M=4, n_train=20000, F=784)),          # feature segments
    ("c4_adjoint", dict(T=7, M=4, n_train=20000, groups=3)),      # output groups
]


@pytest.mark.parametrize("name,over", MODELS, ids=[m[0] + str(i) for i, m in enumerate(MODELS)])
def test_host_tables_under_sanitizers(driver, tmp_path, name, over):
    import paper_2605_04497_amd as q
    wl = synth.make_workload(name, **over)
    line = _run(driver, tmp_path, wl.ensemble)
    assert line.startswith("ok "), line
    kv = dict(tok.split("=") for tok in line.split()[1:])
    info = q.Ensemble(wl.ensemble, host_only=True).info
    assert int(kv["paths"]) == info["n_paths"]
    assert int(kv["elements"]) == info["n_elements"]
    assert int(kv["merged_rows"]) == info["n_value_paths"]
    assert int(kv["segments"]) == info["n_value_segments"]
    # depth-first form: one row per internal node; updates = features split
    # above each internal node other than its own split feature
    ens = wl.ensemble
    n_int, upd = 0, 0
    for t in range(ens.n_trees):
        a = int(ens.tree_offsets[t])
        stack = [(0, frozenset())]
        while stack:
            node, fs = stack.pop()
            g = a + node
            if ens.left[g] < 0:
                continue
            f = int(ens.feature[g])
            n_int += 1
            upd += len(fs - {f})
            stack.append((int(ens.left[g]), fs | {f}))
            stack.append((int(ens.right[g]), fs | {f}))
    assert int(kv["dfs_nodes"]) == n_int and int(kv["dfs_updates"]) == upd
    assert int(kv["dfs_rows"]) % 64 == 0 and int(kv["dfs_rows"]) >= n_int
    assert abs(float(kv["wsum"]) - 7.0) < 1e-13   # each rule's weights sum to 1


def test_malformed_models_under_sanitizers(driver, tmp_path):
    """Cycles, out-of-range children and features, one-child nodes, NaN
    thresholds, negative covers and bad groups are rejected with an error,
    never a memory fault or undefined behaviour."""
    rng = np.random.default_rng(5)
    base = synth.random_small_ensemble(rng, 3, 5, 4)
    cases = []
    for mutate in ("cycle", "child_range", "feature_range", "one_child", "nan_thr",
                   "neg_cover", "group"):
        e = synth.ensembles.Ensemble(base.tree_offsets.copy(), base.left.copy(),
                                     base.right.copy(), base.feature.copy(),
                                     base.threshold.copy(), base.default_left.copy(),
                                     base.cover.copy(), base.value.copy(), base.n_features)
        inner = np.flatnonzero(e.left >= 0)
        i = int(inner[1])
        if mutate == "cycle":
            e.left[i] = 0
        elif mutate == "child_range":
            e.right[i] = 10 ** 6
        elif mutate == "feature_range":
            e.feature[i] = 99
        elif mutate == "one_child":
            e.right[i] = -1
        elif mutate == "nan_thr":
            e.threshold[i] = np.nan
        elif mutate == "neg_cover":
            e.cover[i] = -1.0
        else:
            e = e.with_groups(np.full(e.n_trees, 2), 2)
        cases.append((mutate, e))
    for mutate, e in cases:
        line = _run(driver, tmp_path, e)
        assert line.startswith("error -2") or line.startswith("error -1"), (mutate, line)
