import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


# Long oracle runs that a selected GPU test needs are started as soon as the
# tests are collected, in child processes, so they overlap the GPU session.
ORACLE_JOBS = {
    "test_structured_4096_fifty_trips_vs_oracle": [("structured4096", 0, 50), ("structured4096", 15, 50)],
}


@pytest.hookimpl(trylast=True)
def pytest_collection_modifyitems(session, config, items):
    wanted = [job for it in items for name, jobs in ORACLE_JOBS.items() if it.name == name for job in jobs]
    if wanted:
        sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
        import oracle_jobs

        for job in wanted:
            oracle_jobs.start(*job)
