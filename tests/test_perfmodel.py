"""The memory-bound model of Sec. 6 against the paper's own Tables 1, 3 and 4."""
from paper_0906_1887_amd import perfmodel as pm
from conftest import read_golden

DESIGNS = ["PP", "HG2", "HG4", "GP2", "GP4"]


def _tables():
    bw, theo, actual, time, pct = {}, {}, {}, {}, {}
    for r in read_golden("paper_table1_table4.txt"):
        if r[0] in ("actual", "time", "pct"):
            {"actual": actual, "time": time, "pct": pct}[r[0]][r[1]] = [float(v) for v in r[2:]]
        else:
            bw[r[0]] = float(r[1])
            theo[r[0]] = [float(v) for v in r[2:]]
    return bw, theo, actual, time, pct


def test_theoretical_column():
    bw, theo, _, _, pct = _tables()
    for gpu, M in bw.items():
        for d, printed in zip(DESIGNS, theo[gpu]):
            model = pm.max_signal_bandwidth(M * 1e9, pm.PAPER_EPS[d], 64) / 1e6
            if gpu == "8800GTX" and d == "GP2":
                # printed 6.1 disagrees with the table's own 57% (which needs 5.2)
                assert abs(model - 5.19) < 0.01
                continue
            # two significant figures (one printed value, 3.4 for 3.46, is truncated)
            assert abs(model - printed) <= 0.07 * printed, (gpu, d, model, printed)


def test_actual_column_and_percentages():
    bw, _, actual, time, pct = _tables()
    for gpu in bw:
        for k, d in enumerate(DESIGNS):
            act = 1.28 * 1000.0 / time[gpu][k]            # MHz of signal per second of data
            assert abs(act - actual[gpu][k]) <= 0.051, (gpu, d)
            model = pm.max_signal_bandwidth(bw[gpu] * 1e9, pm.PAPER_EPS[d], 64) / 1e6
            assert abs(100 * act / model - pct[gpu][k]) <= 1.0, (gpu, d, 100 * act / model)


def test_realtime_requirement():
    # 64 inputs at 1.28 MHz: 1.28e6 * 2080 CMAC/s
    assert pm.realtime_cmac_rate(1.28e6, 64) == 1.28e6 * 2080
    assert pm.n_products(64) == 2080


def test_this_build_work():
    assert pm.xengine_cmac(768, 1024, 8000) == 768 * 524800 * 8000
    assert abs(pm.int8_cmac_peak() - 625e12) < 1e6
    # one-pass reads correspond to eps = 2/(N_I+1)
    b1 = pm.global_read_rate(pm.eps_of_one_pass(64), 1.0, 64)
    assert abs(b1 - 64 * 8) < 1e-9
