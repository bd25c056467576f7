import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")
    config.addinivalue_line("markers", "oracle_pool: compares with oracle results computed by the CPU worker pool")


def pytest_collection_finish(session):
    # The full-size parity tests compare with oracle runs of minutes each:
    # start them on CPU workers now, before any test initialises the GPU.
    if any(item.get_closest_marker("oracle_pool") for item in session.items):
        import oracle_pool

        oracle_pool.start()


def pytest_sessionfinish(session, exitstatus):
    import oracle_pool

    oracle_pool.stop()
