"""Host-side logic that needs no GPU: batch-width choice and resume of the
campaign driver, the autotuner's cache keys, the bench's host report and its
one-GPU refusal."""
import json

import pytest


@pytest.fixture(scope="module")
def pkg():
    import paper_2203_09732_amd as m
    return m


def test_widest_batch_is_a_power_of_two_within_limits(pkg):
    from paper_2203_09732_amd import campaign
    for L in (12, 14, 16, 18, 20, 22, 24, 26):
        for want in (1, 2, 3, 5, 8, 17, 32, 100):
            R = campaign.widest_batch(L, want)
            assert R & (R - 1) == 0 and 2 <= R <= campaign.MAX_R
            assert R <= max(2, want)
            # the per-realization field tables of R realizations fit the budget
            assert R == 2 or R * 16 * ((L + 3) // 4) * 8 <= 30 * 1024


def test_campaign_resume_reads_done_indices(pkg, tmp_path):
    from paper_2203_09732_amd import campaign
    p = tmp_path / "r.jsonl"
    assert campaign._done_indices(str(p)) == set()
    with open(p, "w") as fh:
        fh.write(json.dumps({"index": 3}) + "\n")
        fh.write("not json\n")
        fh.write(json.dumps({"index": 7, "L": 14}) + "\n")
    assert campaign._done_indices(str(p)) == {3, 7}


def test_campaign_persistent_mode_chunks_and_resumes(pkg, monkeypatch, tmp_path):
    """The driver's problem-array mode with the library call replaced by a
    stand-in: realizations go in chunks, every one gets a record, and a
    second run over the same results file calls nothing."""
    import numpy as np
    from paper_2203_09732_amd import campaign
    calls = []

    def fake_problems(problems, **kw):
        calls.append([p["L"] for p in problems])
        res = [pkg.ProblemResult(p["L"], 0, np.arange(p["nev"], dtype=float), None,
                                 np.zeros(p["nev"]), np.zeros(p["nev"], complex), 0.5, 20,
                                 p["nev"], 1000, 1e-12, 1.0) for p in problems]
        return 0, res
    monkeypatch.setattr(campaign, "si_lanczos_problems", fake_problems)
    tasks = [campaign.Task(i, (14, 16, 18)[i % 3], 3.0, np.zeros((14, 16, 18)[i % 3]))
             for i in range(5)]
    out = tmp_path / "c.jsonl"
    recs = campaign.run(tasks, 2, results_path=str(out), mode="persistent", chunk=3, log=None)
    assert calls == [[14, 16, 18], [14, 16]]
    assert sorted(r["index"] for r in recs) == list(range(5))
    assert all(r["mode"] == "persistent" and r["nconv"] == 2 for r in recs)
    again = campaign.run(tasks, 2, results_path=str(out), mode="persistent", chunk=3, log=None)
    assert again == [] and len(calls) == 2
    assert campaign._done_indices(str(out)) == set(range(5))


def test_tuner_cache_key_and_default(pkg, monkeypatch, tmp_path):
    from paper_2203_09732_amd import tune
    assert tune._key(22, 32, "fp64") == "L22_R32_fp64"
    cache = tmp_path / "tuning.json"
    cache.write_text(json.dumps({"gfx950": {"L22_R32_fp64": {"lo_bits": 11}}}))
    monkeypatch.setattr(tune, "CACHE", str(cache))
    monkeypatch.setattr(tune, "_arch", lambda: "gfx950")
    assert tune.best_lo_bits(22, 32, "fp64") == 11
    assert tune.best_lo_bits(22, 16, "fp64") == 0       # unknown: library default
    monkeypatch.setattr(tune, "_arch", lambda: "gfx942")
    assert tune.best_lo_bits(22, 32, "fp64") == 0       # other architecture


def test_tuner_schedule_entries(pkg, monkeypatch, tmp_path):
    """Cached schedules: the four knobs of a full entry, zeros (library
    defaults) for entries from before the schedule knobs and for unknown keys;
    apply_schedule hands them to the batch."""
    from paper_2203_09732_amd import tune
    cache = tmp_path / "tuning.json"
    cache.write_text(json.dumps({"gfx950": {
        "L22_R32_fp64": {"lo_bits": 10, "grid": 256, "graph_iters": 8, "dx_group": 4},
        "L26_R16_fp64": {"lo_bits": 13}}}))
    monkeypatch.setattr(tune, "CACHE", str(cache))
    monkeypatch.setattr(tune, "_arch", lambda: "gfx950")
    assert tune.best_schedule(22, 32) == (256, 8, 4)
    assert tune.best_schedule(26, 16) == (0, 0, 0)
    assert tune.best_schedule(18, 32) == (0, 0, 0)

    class FakeBatch:
        def set_schedule(self, *knobs):
            self.knobs = knobs
    fb = FakeBatch()
    tune.apply_schedule(fb, 22, 32)
    assert fb.knobs == (256, 8, 4)


def test_bench_names_the_kernel_it_times():
    import bench
    assert bench.headline_kernel(22, 10, 32) == "k_bapply_staged<22,0>"
    assert bench.headline_kernel(22, 11, 32) == "k_bapply<double,0,false,22,11>"
    assert bench.headline_kernel(22, 10, 16) == "k_bapply<double,0,false,22,10>"


def test_committed_tuning_cache_is_well_formed():
    """Every entry of the committed cache names a split the tuner could pick
    and schedule values the library accepts."""
    import os
    from paper_2203_09732_amd import tune
    data = json.load(open(os.path.join(os.path.dirname(tune.__file__), "tuning.json")))
    for arch, entries in data.items():
        for key, e in entries.items():
            L = int(key.split("_")[0][1:])
            assert e["lo_bits"] in tune.CANDIDATES[L], (key, e)
            assert e.get("grid", 0) in (0,) + tuple(g for g in tune.GRIDS if g)
            assert e.get("graph_iters", 16) in tune.GRAPH_ITERS
            assert e.get("dx_group", 4) in tune.DX_GROUPS


def test_bench_host_report_and_no_projection():
    import bench
    info = bench.host_info()
    assert info["nproc"] >= 1
    assert "blas" in info and "cpu_model" in info
    # every eigenpair figure of the bench line is measured: no projection left
    assert not hasattr(bench, "l22_projection") and not hasattr(bench, "L22_ITERS")


def test_bench_refuses_more_than_one_gpu(capsys):
    import sys

    import bench
    argv = sys.argv
    sys.argv = ["bench.py", "--gpus", "2"]
    try:
        with pytest.raises(SystemExit) as e:
            bench.main()
    finally:
        sys.argv = argv
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().out
