"""The genetic search: pins of its oracle (oracle/ga.py) against the paper's
rules and the generator's published values, then bit-exact parity of the
library's engine (hj_ga_run, host only) with the oracle."""
import ctypes

import numpy as np
import pytest

from oracle import ga


def test_splitmix_published_sequence():
    # SplitMix64 from state 0 (Vigna's reference implementation of Steele et al.)
    assert ga.splitmix_output(0, 0) == 0xE220A8397B1DCDAF
    assert ga.splitmix_output(0, 1) == 0x6E789E6AA1B965F4
    assert ga.splitmix_output(0, 2) == 0x06C45D188009454F


def test_uniform_range_and_moments():
    u = np.array([ga.uniform(7, 3, n) for n in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01 and abs(u.var() - 1 / 12) < 0.005


def test_fitness_is_inverse_square_root_of_time():
    assert ga.fitness(4.0) == 0.5
    assert ga.fitness(0.01) == 10.0


def test_roulette_picks_in_proportion_to_fitness():
    fit = [1.0, 2.0, 3.0, 4.0]
    total = sum(fit)
    counts = np.zeros(4)
    for n in range(40000):
        counts[ga.roulette(fit, total, ga.uniform(1, 9, n))] += 1
    np.testing.assert_allclose(counts / counts.sum(), np.array(fit) / total, atol=0.01)
    assert ga.roulette(fit, total, 0.0) == 0
    assert ga.roulette(fit, total, 1.0 - 2 ** -53) == 3


def random_table(L, seed):
    rng = np.random.default_rng(seed)
    return list(rng.uniform(0.01, 2.0, 2 ** L))


def test_elitism_keeps_the_best_and_best_never_worsens():
    L, M, T = 8, 8, 12
    tab = random_table(L, 1)
    _, best_t, _, hist = ga.run(L, M, T, 42, 0.9, 0.05, lambda g: tab[g])
    prev_best = None
    for g in range(T):
        gen_best = min(tab[x] for x in hist[g])
        if g > 0:
            elite = min(hist[g - 1], key=lambda x: (tab[x], hist[g - 1].index(x)))
            assert hist[g][0] == elite
            assert gen_best <= prev_best
        prev_best = gen_best
    assert best_t == min(tab[x] for h in hist for x in h)


def test_without_crossover_or_mutation_only_copies():
    L, M, T = 8, 10, 8
    tab = random_table(L, 2)
    _, _, _, hist = ga.run(L, M, T, 5, 0.0, 0.0, lambda g: tab[g])
    for g in range(1, T):
        assert set(hist[g]) <= set(hist[g - 1])


def test_crossover_children_are_one_cut_splices_of_parents():
    L, M, T = 8, 10, 6
    tab = random_table(L, 3)
    _, _, _, hist = ga.run(L, M, T, 11, 1.0, 0.0, lambda g: tab[g])
    full = (1 << L) - 1
    for g in range(1, T):
        prev = hist[g - 1]
        for c in hist[g][1:]:
            ok = any(((a & ((1 << p) - 1)) | (b & ~((1 << p) - 1) & full)) == c
                     for a in prev for b in prev for p in range(1, L))
            assert ok, (g, c)


def test_full_mutation_complements_parents():
    L, M, T = 8, 6, 5
    tab = random_table(L, 4)
    _, _, _, hist = ga.run(L, M, T, 13, 0.0, 1.0, lambda g: tab[g])
    full = (1 << L) - 1
    for g in range(1, T):
        for c in hist[g][1:]:
            assert (c ^ full) in hist[g - 1]


def test_failures_count_as_a_thousand_seconds():
    L = 4
    tab = [float("nan"), -1.0, 5000.0] + [2.0] * (2 ** L - 3)
    seen = {}

    def t(g):
        seen[g] = True
        return tab[g]
    best, best_t, _, _ = ga.run(L, 6, 6, 3, 0.9, 0.05, t)
    assert best_t == 2.0 and best >= 3


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_reaches_the_optimum_of_a_simple_landscape(seed):
    L = 10
    target = 0b1011001110
    tab = [1.0 + bin(g ^ target).count("1") for g in range(2 ** L)]
    best, best_t, evals, _ = ga.run(L, 20, 40, seed, 0.9, 0.05, lambda g: tab[g])
    assert best == target and best_t == 1.0
    assert evals < 2 ** L


# ---- parity of the library's engine with the oracle -------------------------

@pytest.fixture(scope="module")
def lib():
    from paper_2002_12115_amd import hj
    lib = hj.load()
    lib.hj_ga_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_ulonglong, ctypes.c_double,
                              ctypes.c_double, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint),
                              ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
    lib.hj_ga_run.restype = ctypes.c_int
    return lib


CASES = [(10, 10, 10, 2002, 0.9, 0.05), (10, 7, 9, 1, 0.9, 0.05), (8, 16, 20, 7, 0.6, 0.2),
         (12, 12, 12, 123456789, 1.0, 0.01), (5, 3, 4, 0, 0.0, 0.0), (1, 4, 5, 9, 0.9, 0.5),
         (16, 10, 10, 2 ** 63 + 5, 0.9, 0.05)]


@pytest.mark.parametrize("L,M,T,seed,pc,pm", CASES)
def test_library_engine_matches_oracle_bitwise(lib, L, M, T, seed, pc, pm):
    tab = np.asarray(random_table(L, seed % 1000), dtype=np.float64)
    tab[::7] = 5000.0          # some failed measurements
    best = ctypes.c_uint()
    best_t = ctypes.c_double()
    evals = ctypes.c_int()
    hist = np.zeros(M * T, dtype=np.uint32)
    rc = lib.hj_ga_run(L, M, T, seed, pc, pm, tab.ctypes.data, ctypes.byref(best), ctypes.byref(best_t),
                       hist.ctypes.data, ctypes.byref(evals))
    assert rc == 0
    obest, obest_t, oevals, ohist = ga.run(L, M, T, seed, pc, pm, lambda g: float(tab[g]))
    assert hist.reshape(T, M).tolist() == ohist
    assert best.value == obest and best_t.value == obest_t and evals.value == oevals


def test_library_engine_rejects_bad_arguments(lib):
    tab = np.ones(4)
    assert lib.hj_ga_run(0, 4, 4, 1, 0.9, 0.05, tab.ctypes.data, None, None, None, None) == -1
    assert lib.hj_ga_run(2, 4, 4, 1, 1.5, 0.05, tab.ctypes.data, None, None, None, None) == -1
    assert lib.hj_ga_run(2, 4, 4, 1, 0.9, 0.05, None, None, None, None, None) == -1


def test_gene_decoding(lib):
    from paper_2002_12115_amd import hj
    lib.hj_gene_config.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_uint, ctypes.POINTER(hj.Config)]
    lib.hj_gene_config.restype = ctypes.c_int
    c = hj.Config()

    def dec(dtype, gene, batch=0, shape=(130, 130, 258)):
        assert lib.hj_gene_config(dtype, *shape, batch, gene, ctypes.byref(c)) == 0
        return c.as_dict()
    two = 1 << 10
    # one iteration: march, bj 4, vec 2, chunk choice 0, non-temporal, no remap
    d = dec(0, 1 | (2 << 1) | (1 << 3) | (1 << 8))
    assert (d["kernel"], d["bj"], d["vec"], d["nontemporal"], d["xcd_remap"], d["tsteps"]) == (1, 4, 2, 1, 0, 1)
    assert dec(0, 1 | (1 << 9))["xcd_remap"] == 1
    # every gene names a configuration, for both dtypes, solves and batches
    for dtype in (0, 1):
        for batch in (0, 1):
            for g in range(2 ** 11):
                d = dec(dtype, g, batch, shape=(0, 0, 0) if batch else (130, 130, 258))
                assert d["tsteps"] == (2 if g & two else 1)
                if d["tsteps"] == 2:
                    # the settings the exhaustive search keeps for two-iteration passes
                    assert d["kernel"] == 1 and d["nontemporal"] == 0 and d["xcd_remap"] == 1
                    assert d["persistent"] == 0 and d["reread"] == (g >> 3) & 1
                    if batch:
                        assert d["ichunk"] == (8, 12, 16, 24, 32, 48, 64, 128)[(g >> 5) & 7]
                        assert d["vec"] == (4 if g & 1 else 1)
                    else:
                        assert d["vec"] == (2 if g & 1 else 1)
                    # bits 4, 8 and 9 are unused here
                    assert d == dec(dtype, g ^ (1 << 4) ^ (1 << 8) ^ (1 << 9), batch,
                                    shape=(0, 0, 0) if batch else (130, 130, 258))
                else:
                    assert d["reread"] == 0
                    if batch:
                        assert d["kernel"] in (1, 2) and d["xcd_remap"] == 0
                        assert d["persistent"] == (g >> 9) & 1
                        assert d["ichunk"] == 2 << ((g >> 5) & 3)
                    elif d["kernel"] != 1:
                        assert d["xcd_remap"] == 0 and d["vec"] == 1
    # folded codes: vec code 2 is 1 for FP64 and 4 for FP32; direct reads bj 1 as 2
    assert dec(0, 1 | (2 << 3))["vec"] == 1 and dec(1, 1 | (2 << 3))["vec"] == 4
    assert dec(0, 0)["bj"] == 2 and dec(0, 0)["kernel"] == 0
    d = dec(0, 1 << 3)                                  # bit 0 clear, bit 3 set: the flat kernel
    assert (d["kernel"], d["tsteps"], d["bj"]) == (2, 1, 2)
    # a flat run too wide for the grid folds onto the march kernel
    assert dec(0, (1 << 3) | (3 << 1), shape=(5, 6, 900))["kernel"] == 1
    # two iterations: bj codes per row layout
    assert [dec(0, two | (b << 1))["bj"] for b in range(4)] == [4, 6, 8, 14]
    assert [dec(0, two | 1 | (b << 1))["bj"] for b in range(4)] == [4, 6, 8, 12]
    assert [dec(1, two | 1 | (b << 1), batch=1, shape=(0, 0, 0))["bj"] for b in range(4)] == [6, 14, 22, 30]
    # the 64-cell rows tile a 256-wide interior in 4: bj 8 fits 256 workgroups in 4 x 16 x 4 chunks of 32
    assert dec(0, two | 1 | (2 << 1))["ichunk"] == 32
    # their chunks: the longest within 256, 512, ... workgroups (5 x 16 tiles of 62-cell rows, bj 8)
    fch = [dec(0, two | (2 << 1) | (sel << 5))["ichunk"] for sel in range(8)]
    assert fch[:4] == [43, 22, 15, 11]
    for sel, wg in enumerate((256, 512, 768, 1024, 1536, 2048, 4096, 16384)):
        assert 80 * -(-128 // fch[sel]) <= wg
    # batch: bit 9 is the persistent grid, the chunk is 2 << (bits 5-6)
    d = dec(1, 1 | (1 << 1) | (2 << 5) | (1 << 9), batch=1, shape=(0, 0, 0))
    assert (d["kernel"], d["persistent"], d["ichunk"], d["xcd_remap"]) == (1, 1, 8, 0)
    assert dec(1, (2 << 1) | (2 << 5), batch=1, shape=(0, 0, 0))["kernel"] == 2
    # one-iteration chunk choices shrink as the workgroup target grows
    ch = [dec(0, 1 | (2 << 1) | (sel << 5))["ichunk"] for sel in range(4)]
    assert ch == sorted(ch, reverse=True)
    assert lib.hj_gene_config(5, 130, 130, 258, 0, 0, ctypes.byref(c)) == -3
