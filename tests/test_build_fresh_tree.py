"""__graft_entry__.build() on a tree without a built library: it must compile libfof.so and
then import the package (the package itself refuses to import without the library)."""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_build_from_a_tree_without_the_library(tmp_path):
    for d in ("paper_2510_26851_amd", "include", "oracle", "workloads"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d,
                        ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    shutil.copy(os.path.join(ROOT, "__graft_entry__.py"), tmp_path)
    assert not (tmp_path / "paper_2510_26851_amd" / "libfof.so").exists()
    r = subprocess.run([sys.executable, "-c",
                        "import __graft_entry__ as g; g.build(); "
                        "import paper_2510_26851_amd as p; print('imported', p.Plan.__name__)"],
                       cwd=tmp_path, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "imported Plan" in r.stdout
    assert (tmp_path / "paper_2510_26851_amd" / "libfof.so").exists()
