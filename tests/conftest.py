import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle checks that take more than a few seconds")


def pytest_sessionstart(session):
    # a planted oracle mistake for the mutation test's child runs (CPU only; see oracle_mutations)
    name = os.environ.get("FGFRFT_ORACLE_MUTATION")
    if name:
        import oracle_mutations
        oracle_mutations.apply(name)
