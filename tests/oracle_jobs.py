"""Oracle runs started in child processes while the GPU tests run (test
infrastructure).  A long FP64 oracle run (50 round trips of a 4096^2 cavity
take minutes on one core) is launched when its test is collected and joined
by that test, so the CPU work overlaps the rest of the GPU session.

Run as a script: oracle_jobs.py WORKLOAD INDEX TRIPS OUTDIR writes
E.npy, N.npy and trace.npy of the oracle after TRIPS round trips of cavity
INDEX of the workload (structured4096) to OUTDIR, then a file named done.
"""
import atexit
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_jobs = {}


@atexit.register
def _stop_unfinished():
    for proc, _, _ in _jobs.values():
        if proc.poll() is None:
            proc.kill()


def start(workload: str, index: int, trips: int):
    key = (workload, index, trips)
    if key not in _jobs:
        out = tempfile.mkdtemp(prefix="oracle_%s_%d_" % (workload, index))
        log = open(os.path.join(out, "log"), "w")
        proc = subprocess.Popen([sys.executable, os.path.abspath(__file__), workload, str(index), str(trips), out],
                                stdout=log, stderr=subprocess.STDOUT, cwd=ROOT)
        _jobs[key] = (proc, out, time.time())
    return _jobs[key]


def result(workload: str, index: int, trips: int, timeout: float = 1200.0):
    """(E, N, trace) of a started job, waiting for it to finish."""
    import numpy as np

    proc, out, _ = start(workload, index, trips)
    proc.wait(timeout=timeout)
    if proc.returncode != 0 or not os.path.exists(os.path.join(out, "done")):
        with open(os.path.join(out, "log")) as f:
            raise RuntimeError("oracle job %s failed:\n%s" % ((workload, index, trips), f.read()[-2000:]))
    return tuple(np.load(os.path.join(out, n + ".npy")) for n in ("E", "N", "trace"))


def _main(argv):
    sys.path.insert(0, ROOT)
    import numpy as np

    import oracle
    from paper_1410_2855_amd.inputs import initial_state, oracle_params, structured_4096

    workload, index, trips, out = argv[1], int(argv[2]), int(argv[3]), argv[4]
    if workload != "structured4096":
        raise SystemExit("unknown workload %s" % workload)
    cav = structured_4096()[index]
    t0 = time.time()
    e, n, tr = oracle.run(oracle_params(cav), *initial_state(cav), trips)
    np.save(os.path.join(out, "E.npy"), e)
    np.save(os.path.join(out, "N.npy"), n)
    np.save(os.path.join(out, "trace.npy"), tr)
    open(os.path.join(out, "done"), "w").write("%.1f s\n" % (time.time() - t0))
    print("oracle %s[%d], %d trips: %.1f s" % (workload, index, trips, time.time() - t0), flush=True)


if __name__ == "__main__":
    _main(sys.argv)
