"""Host-side logic that needs no GPU: batch grouping, the plane-wave count,
autotune candidates, the batched workload draws and the benchmark's byte model."""
import itertools
import math

import numpy as np

from paper_1811_11679_amd import autotune, batch, workloads


def test_plane_wave_counts_are_lattice_point_counts():
    # integer vectors with |n|^2 <= c: 1 + 6 + 12 + 8 + 6 + 24 + 24 + ... by shells
    def brute(c):
        m = int(math.isqrt(c)) + 1
        return sum(1 for v in itertools.product(range(-m, m + 1), repeat=3) if sum(x * x for x in v) <= c)
    for c, n in [(0, 1), (1, 7), (2, 19), (3, 27), (5, 57), (9, 123), (14, 251)]:
        assert batch.n_plane_waves(c) == n == brute(c)


def test_key_words_round_up_to_a_power_of_two():
    assert batch.key_words(dict(kind="hubbard", n_sites=8)) == 1
    assert batch.key_words(dict(kind="hubbard", n_sites=32)) == 1
    assert batch.key_words(dict(kind="hubbard", n_sites=33)) == 2
    assert batch.key_words(dict(kind="ueg", ecut_n2=2)) == 1    # 38 spin-orbitals
    assert batch.key_words(dict(kind="ueg", ecut_n2=5)) == 2    # 114
    assert batch.key_words(dict(kind="ueg", ecut_n2=9)) == 4    # 246
    assert batch.key_words(dict(kind="ueg", ecut_n2=14)) == 8   # 502
    assert batch.key_words(dict(kind="molecular", n_orb=100)) == 4  # 200 -> 4 words


def test_autotune_candidates_are_cu_multiples_and_keep_the_current():
    c = autotune.candidates(256, 999)
    assert 999 in c and c == sorted(set(c))
    assert all(x % 256 == 0 for x in c if x != 999)
    assert min(c) == 256 and max(c) == 256 * 16


def test_batched_workload_draws_are_seeded_and_in_range():
    a, b = workloads.batch64(), workloads.batch64()
    assert len(a) == 64
    assert [x[1]["target_population"] for x in a] == [x[1]["target_population"] for x in b]
    for r, (sysd, q) in enumerate(a):
        assert sysd["kind"] == "ueg" and sysd["n_alpha"] == sysd["n_beta"] == 7
        assert sysd["rs"] in (0.5, 1.0, 2.0, 4.0)
        assert batch.n_plane_waves(sysd["ecut_n2"]) in (19, 27, 57, 123)
        assert 1e5 <= q["target_population"] <= 2e6
        assert q["tau"] == 0.002 * min(1.0, sysd["rs"] ** 2)
        assert q["replica_id"] == r


def test_byte_model_counts_the_moved_fields():
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location("bench", os.path.join(os.path.dirname(__file__), "..", "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    prev = dict(n_occupied=1000)
    cur = dict(n_occupied=1100, n_spawned=300, n_spawn_events=200)
    b1 = bench.algorithmic_bytes(prev, cur, 2)
    # one instance, W = 2, no deterministic space: main read 16+4+8, distinct 8+16+8+4, output 16+4+8+8+1
    assert b1["merge"] == 1000 * 28 + 200 * 36 + 1100 * 37
    # spawn: parent key, population, attempt offset; per spawn sort key + key words + amplitude word
    assert b1["spawn"] == 1000 * (16 + 4 + 8) + 300 * (8 + 16 + 8)
    b2 = bench.algorithmic_bytes(prev, cur, 2, ds_active=True, instances=4)
    assert b2["merge"] - b1["merge"] == 1000 * 12 + 1100 * 12
    b8 = bench.algorithmic_bytes(prev, cur, 8)
    assert b8["merge"] - bench.algorithmic_bytes(prev, cur, 8, instances=2)["merge"] == 0  # long keys keep sort keys
    assert np.isclose(b1["sort_pass1"], 300 * 24)
    # CCMC at CCSD on 14 electrons: sizes 2, 3, 4 with p = 1/2, 1/4, 1/4 (mean 2.75);
    # n_c = ceil(N_ex 2^-8) with N_ex = N_w - |N_0| of the previous iteration
    prev_c = dict(n_occupied=1000, n_walkers_units=256 * 500 + 100, ref_pop_units=-100)
    cur_c = dict(n_occupied=1000, n_spawned=300, n_spawn_events=200, n_cluster_spawns=40)
    bc = bench.algorithmic_bytes(prev_c, cur_c, 2, ccmc=(2, 14, 8))
    assert np.isclose(bc["ccmc_clusters"], 1000 * (16 + 4 + 8) + 500 * 2.75 * (16 + 4) + 40 * (8 + 16 + 8))
    assert "ccmc_clusters" not in b1
