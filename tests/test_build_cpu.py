"""The build entry point on a tree with no built libraries (the state of a
fresh checkout, where the .so files are not in version control): build()
must compile libmbmd.so and the oracle and then import the package.  The
package refuses to import without its library, so build() must not import
it before building."""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_build_from_a_tree_without_libraries(tmp_path):
    dst = tmp_path / "tree"
    shutil.copytree(ROOT, dst, ignore=shutil.ignore_patterns(
        "*.so", "*.o", "_build", "_work", "gpurun_out", ".git", "__pycache__", ".pytest_cache"))
    assert not (dst / "paper_1610_03343_amd" / "libmbmd.so").exists()
    r = subprocess.run([sys.executable, "-c", "import __graft_entry__ as g; g.build()"],
                       cwd=dst, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-2000:]
    assert (dst / "paper_1610_03343_amd" / "libmbmd.so").exists()
    assert (dst / "oracle" / "liboracle.so").exists()
