"""Committed code reads nothing from the private working folder, and only
tests, the smoke check and the bench's CPU baseline touch the oracle."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CODE = (".py", ".hip", ".h", ".cpp", ".c", ".sh", ".ini", ".toml", ".cfg")


def _files():
    for top in ("paper_2201_10022_amd", "oracle", "scenegen", "tests", "include"):
        for dirpath, dirs, files in os.walk(os.path.join(ROOT, top)):
            dirs[:] = [d for d in dirs if not d.startswith(("_build", "__pycache__", "."))]
            for f in files:
                if f.endswith(CODE):
                    yield os.path.join(dirpath, f)
    for f in ("bench.py", "__graft_entry__.py", "pytest.ini"):
        yield os.path.join(ROOT, f)


def test_no_reads_of_the_private_working_folder():
    me = os.path.abspath(__file__)
    bad = re.compile(r"(^|[^\w])_work/")
    seen = 0
    for path in _files():
        if os.path.abspath(path) == me or not os.path.exists(path):
            continue
        seen += 1
        src = open(path, errors="replace").read()
        assert not bad.search(src), path
    assert seen > 20


def test_oracle_used_only_by_tests_smoke_and_cpu_baseline():
    imp = re.compile(r"^\s*(import oracle|from oracle)", re.M)
    for path in _files():
        rel = os.path.relpath(path, ROOT)
        if rel.startswith(("tests", "oracle")) or rel in ("bench.py", "__graft_entry__.py"):
            continue
        if os.path.exists(path):
            assert not imp.search(open(path, errors="replace").read()), rel
