"""The product path has no CPU fallback: importing the package without its HIP
library raises ImportError naming the missing library.  Checked in a
subprocess on a copy of the package's Python files in a scratch directory, so
the built library of the repository is not touched."""

import glob
import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_import_fails_without_the_hip_library():
    d = tempfile.mkdtemp()
    try:
        pk = os.path.join(d, "paper_1012_2677_amd")
        os.makedirs(pk)
        for f in glob.glob(os.path.join(ROOT, "paper_1012_2677_amd", "*.py")):
            shutil.copy(f, pk)
        assert not os.path.exists(os.path.join(pk, "libmd355.so"))
        r = subprocess.run([sys.executable, "-c", "import paper_1012_2677_amd"], cwd=d, capture_output=True,
                           text=True, env=dict(os.environ, PYTHONPATH=d), timeout=300)
        assert r.returncode != 0
        assert "ImportError" in r.stderr
        assert "libmd355.so is missing" in r.stderr
    finally:
        shutil.rmtree(d)
