"""Autotuning with on-disk caches: the library's SpMV slab shape (cached per layout and
device in RAFEM_TUNE_CACHE) and the mixed refinement's inner tolerance and restart mode
(paper_2409_13036_amd.tune, cached in a JSON file).  A cached choice is reused without
timing, and a tuned shape never changes a result."""
import os

import numpy as np
import pytest

import rafem_inputs as ri
from gpu_helpers import to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def test_spmv_shape_cache_is_written_then_reused(torch_cuda, tmp_path, monkeypatch):
    from paper_2409_13036_amd.sim import DeviceProblem
    cache = tmp_path / "spmv_tune.txt"
    monkeypatch.setenv("RAFEM_TUNE_CACHE", str(cache))
    p = ri.make_problem("hex", 21, 3)
    out = []
    for k in range(2):
        dp = DeviceProblem(p)
        dp.step(1e-12, "mixed")
        st = dp.mesh.stats()
        out.append((st.tuned_from_cache, st.slabs_per_block, st.slabs_per_block32,
                    st.launch_bound, st.launch_bound32, to_host(dp.T), to_host(dp.V)))
        dp.close()
    lines = cache.read_text().split("\n")
    print(f"[tune] cache: {lines[0]}", flush=True)
    assert out[0][0] == 0 and out[1][0] == 1       # timed first, then read from the cache
    assert out[0][1:5] == out[1][1:5]
    assert out[0][3] in (1, 6) and out[0][4] in (1, 6)
    assert len(lines[0].split()) == 9
    assert len([l for l in lines if l.strip()]) == 1
    assert np.array_equal(out[0][5], out[1][5]) and np.array_equal(out[0][6], out[1][6])
    # a line of the right key with a launch bound the library does not build (3) is
    # ignored: the shapes are timed again and a valid line is appended
    f = lines[0].split()
    cache.write_text(" ".join(f[:7] + ["3", "3"]) + "\n")
    dp = DeviceProblem(p)
    dp.step(1e-12, "mixed")
    st = dp.mesh.stats()
    assert st.tuned_from_cache == 0 and st.launch_bound in (1, 6)
    dp.close()
    lines = [l for l in cache.read_text().split("\n") if l.strip()]
    assert len(lines) == 2 and lines[1].split()[0] == f[0] and lines[1].split()[7] in ("1", "6")


def test_mixed_tuner_picks_a_candidate_and_caches_it(torch_cuda, tmp_path):
    from paper_2409_13036_amd.sim import DeviceProblem
    from paper_2409_13036_amd.tune import tune_mixed
    path = str(tmp_path / "mixed.json")
    p = ri.make_problem("hex", 21, 4, steps=6)
    dp = DeviceProblem(p)
    dp.extrapolate = True
    cands = ((1e-4, 0), (1e-3, 0), (1e-4, 1))
    first = tune_mixed(dp, warmup=1, steps=2, candidates=cands, path=path)
    again = tune_mixed(dp, warmup=1, steps=2, candidates=cands, path=path)
    print(f"[tune] mixed: {first}", flush=True)
    assert not first["cached"] and again["cached"]
    assert (first["inner_tol"], first["restart_inner"]) in cands
    assert (again["inner_tol"], again["restart_inner"]) == (first["inner_tol"], first["restart_inner"])
    assert len(first["timings"]) == len(cands)
    # the chosen setting solves the step to the FP64 path's answer
    dp.reset()
    dp.step(1e-13, "mixed", inner_tol=first["inner_tol"], restart_inner=first["restart_inner"])
    Tm = to_host(dp.T)
    dp.reset()
    dp.step(1e-13, "fp64")
    T6 = to_host(dp.T)
    dp.close()
    assert np.linalg.norm(Tm - T6) <= 1e-8 * np.linalg.norm(T6)
    assert os.path.exists(path)


def _far_swaps(p, dist):
    from paper_2409_13036_amd.sim import reorder_nodes
    order = np.arange(p.n_nodes)
    a = np.sort(np.random.default_rng(7).choice(np.arange(200, p.n_nodes - dist), 6,
                                                replace=False))
    order[a], order[a + dist] = a + dist, a
    return reorder_nodes(p, order)


def _shuffled(p):
    from paper_2409_13036_amd.sim import reorder_nodes
    return reorder_nodes(p, np.random.default_rng(5).permutation(p.n_nodes))


@pytest.mark.parametrize("mesh", ["hex21", "tet13", "hex41-shuffled", "hex41-far-swaps"])
def test_streamed_value_loads_give_the_same_bits(torch_cuda, tmp_path, monkeypatch, mesh):
    """The SpMV configuration read from the cache is used as written, and neither the
    nontemporal reads of the matrix values (the autotuner's choice for matrices beyond the
    Infinity Cache), whole or past a prefix read with ordinary loads, nor the kernels' launch
    bound (1 or 6 resident workgroups per CU) changes a bit of a coupled step, in FP64 and
    mixed precision, on every slab kind: shared offset lists and 16-bit offsets (hex21,
    tet13), 32-bit columns (shuffled), and both widths in one layout (nodes swapped 40,000
    positions apart)."""
    from paper_2409_13036_amd.sim import DeviceProblem
    cache = tmp_path / "spmv_tune.txt"
    monkeypatch.setenv("RAFEM_TUNE_CACHE", str(cache))
    p = {"hex21": lambda: ri.make_problem("hex", 21, 3),
         "tet13": lambda: ri.make_problem("tet", 13, 3),
         "hex41-shuffled": lambda: _shuffled(ri.make_problem("hex", 41, 3)),
         "hex41-far-swaps": lambda: _far_swaps(ri.make_problem("hex", 41, 3), 40000)}[mesh]()
    dp = DeviceProblem(p)
    dp.step(1e-12, "mixed")
    half = int(dp.mesh.stats().value_slots) // 2
    dp.close()
    key, spb64, spb32 = cache.read_text().split()[:3]
    out = {}
    for nt, res, mb in ((0, 0, 1), (1, 0, 6), (1, half, 1), (0, 0, 6)):
        cache.write_text(f"{key} {spb64} {spb32} {nt} {nt} {res} {res} {mb} {mb}\n")
        dp = DeviceProblem(p)
        states = []
        for prec in ("fp64", "mixed"):
            dp.reset()
            for _ in range(2):
                dp.step(1e-12, prec)
            states.append((to_host(dp.T), to_host(dp.V)))
        st = dp.mesh.stats()
        if mesh == "hex41-far-swaps":
            assert st.int16_columns == 1 and st.int32_column_slabs > 0
        if mesh == "hex41-shuffled":
            assert st.int16_columns == 0
        assert st.tuned_from_cache == 1
        assert st.streamed_values == nt and st.streamed_values32 == nt
        assert st.resident_slots == res and st.resident_slots32 == res
        assert st.launch_bound == mb and st.launch_bound32 == mb
        out[(nt, res, mb)] = states
        dp.close()
    ref = out[(0, 0, 1)]
    for key2, states in out.items():
        for (Ta, Va), (Tb, Vb) in zip(ref, states):
            assert np.array_equal(Ta, Tb) and np.array_equal(Va, Vb), key2
