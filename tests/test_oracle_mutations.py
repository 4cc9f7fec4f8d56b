"""The oracle's pins catch plausible mistakes: each mutation in oracle_mutations (one slip in
one routine: a dropped term, a wrong sign or index, a missing conjugate) is planted in a child
pytest run of the pin suite, which must then fail.  CPU only."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
from oracle_mutations import MUTATIONS  # noqa: E402


def _run(name):
    env = dict(os.environ, FGFRFT_ORACLE_MUTATION=name, OMP_NUM_THREADS="2", OPENBLAS_NUM_THREADS="2",
               MKL_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle_pins.py"), "-x", "-q",
                        "-p", "no:cacheprovider", "-m", "not gpu"], env=env, capture_output=True, text=True,
                       timeout=600)
    return name, r.returncode, r.stdout[-2000:]


@pytest.mark.timeout(900)
def test_every_planted_oracle_mistake_fails_a_pin():
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(_run, sorted(MUTATIONS)))
    survivors = [(n, out) for n, rc, out in results if rc == 0]
    assert not survivors, "mutations no pin catches: " + ", ".join(n for n, _ in survivors)
    for n, rc, out in results:
        assert rc == 1, (n, rc, out)     # a failing test (not a crash of the runner)
