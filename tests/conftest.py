import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def batch64():
    """The 64-frame batch workload (uneven frames: 640x360 / 1280x720 /
    1920x1080, N log-uniform in [5e4, 2e6], seed 1003) and the plain oracle's
    result for every frame, computed once per session.  The oracle runs one
    frame per host thread (its C entry point releases the interpreter lock);
    each frame is still sorted by the single-threaded plain oracle."""
    import concurrent.futures

    import oracle
    import synth

    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        frames = list(ex.map(lambda f: synth.batch_frame(synth.SEED_BASE + 3, f), range(64)))
        refs = list(ex.map(lambda fr: oracle.sort_frame(fr[0], fr[1], fr[2], stages=False), frames))
    for r in refs:
        assert r.status == oracle.OK
    return frames, refs
