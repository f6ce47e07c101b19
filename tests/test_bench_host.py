"""bench.py's command-line contract on the host (no GPU is touched)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env={**os.environ, "HIP_VISIBLE_DEVICES": ""})


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_the_contract_options():
    r = _run("--help")
    assert r.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--workload", "--batch", "--prec"):
        assert opt in r.stdout


def test_traffic_summary_weights_the_forward_builds(tmp_path):
    """profiling traffic: per-dispatch bytes scaled by the copy calibration,
    and the forward step over all its builds weighted by dispatches."""
    def reduced(path, rows):
        with open(path, "w") as f:
            f.write("Kernel_Name,Counter_Name,Counter_Sum,Dispatches\n")
            for k, c, v, n in rows:
                f.write(f"\"{k}\",{c},{v},{n}\n")
    fe, wr, cf, cw = (tmp_path / n for n in ("f.csv", "w.csv", "cf.csv", "cw.csv"))
    reduced(fe, [("void swc::k_fwd<double, false>(swc::Tab)", "FETCH_SIZE", 200.0, 2),
                 ("void swc::k_fwd_ho<double>(swc::Tab)", "FETCH_SIZE", 1800.0, 6)])
    reduced(wr, [("void swc::k_fwd<double, false>(swc::Tab)", "WRITE_SIZE", 20.0, 2),
                 ("void swc::k_fwd_ho<double>(swc::Tab)", "WRITE_SIZE", 60.0, 6)])
    # a 1 MiB copy that FETCH_SIZE counts at half its bytes and WRITE_SIZE at all of them
    reduced(cf, [("copy_kernel", "FETCH_SIZE", 512.0, 1)])
    reduced(cw, [("copy_kernel", "WRITE_SIZE", 1024.0, 1)])
    r = subprocess.run([sys.executable, "-m", "paper_2301_05726_amd.profiling", "traffic", "--fetch", str(fe),
                        "--write", str(wr), "--cal-fetch", str(cf), "--cal-write", str(cw), "--cal-mib", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    vals = {p[1]: float(p[2]) for p in (l.split() for l in r.stdout.splitlines()) if p and p[0] == "traffic_kib"}
    assert vals["k_fwd"] == 2 * 100.0 + 10.0        # per dispatch: fetch x 2 + write x 1
    assert vals["k_fwd_ho"] == 2 * 300.0 + 10.0
    assert vals["k_fwd_step"] == (2 * 210.0 + 6 * 610.0) / 8
    assert "k_rev_step" not in vals
