"""The rocprofv3 summaries under profiles/ quote the exact commands they come
from: every such command runs a committed bench.py with options that its
command line accepts."""
import glob
import importlib.util
import os
import shlex

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _parser():
    spec = importlib.util.spec_from_file_location("bench_cli", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.build_parser()


def _commands(path):
    """bench.py argument lists of the indented (code block) commands."""
    text = open(path).read().replace("\\\n", " ")
    out = []
    for line in text.splitlines():
        if line.startswith("    ") and "python bench.py" in line:
            out.append(shlex.split(line.split("python bench.py", 1)[1]))
    return out


def test_profile_commands_parse():
    ap = _parser()
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))
    assert paths
    total = 0
    for path in paths:
        cmds = _commands(path)
        assert cmds, "%s quotes no bench.py command" % os.path.basename(path)
        for args in cmds:
            ap.parse_args(args)  # an unknown option exits (SystemExit fails the test)
        total += len(cmds)
    assert total >= len(paths)
