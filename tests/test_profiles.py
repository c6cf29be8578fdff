"""The profiler summaries under profiles/ stay reproducible: every one quotes the commands that
made it, those commands run committed scripts only (no working files), bench.py's own parser
accepts their arguments, and each counter run stays within the per-block counter limits of one
rocprofv3 pass (4 TCC, 8 SQ counters).  CPU only."""
import glob
import os
import re
import shlex
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))

# hardware counters behind the derived ones used here, and the blocks they occupy
TCC_COST = {"FETCH_SIZE": 3, "WRITE_SIZE": 2}


def _commands(path):
    """rocprofv3 command lines, with the shell variables the summary sets (NAME="...") expanded."""
    env, cmds = {}, []
    for ln in open(path):
        ln = ln.strip()
        m = re.fullmatch(r'([A-Z][A-Z0-9_]*)="([^"]*)"', ln)
        if m:
            env[m.group(1)] = m.group(2)
        elif "rocprofv3" in ln and " -- " in ln:
            ln = re.sub(r"\$([A-Z][A-Z0-9_]*)\b", lambda m: env.get(m.group(1), m.group(0)), ln)
            cmds.append(ln)
    return cmds


def _tracked(rel):
    out = subprocess.run(["git", "ls-files", "--error-unmatch", rel], cwd=ROOT,
                         capture_output=True, text=True)
    return out.returncode == 0


def test_every_profile_quotes_its_commands():
    assert PROFILES
    for path in PROFILES:
        assert _commands(path), os.path.basename(path)


@pytest.mark.parametrize("path", PROFILES, ids=[os.path.basename(p) for p in PROFILES])
def test_profile_commands_run_committed_files(path):
    import bench
    parser = bench.make_parser()
    for line in _commands(path):
        tool, prog = line.split(" -- ", 1)
        argv = shlex.split(prog)
        assert argv[0] == "python3", line
        script = argv[1].replace("$REPO/", "")
        assert not script.startswith("_work"), line
        assert _tracked(script), f"{script} is not a committed file"
        if script == "bench.py":
            parser.parse_args(argv[2:])
        # one counter pass: at most 4 TCC counters (a derived counter counts its inputs)
        targs = shlex.split(tool)
        if "--pmc" in targs:
            i = targs.index("--pmc") + 1
            names = []
            while i < len(targs) and not targs[i].startswith("-"):
                names.append(targs[i])
                i += 1
            assert names, line
            tcc = sum(TCC_COST.get(n, 1 if n.startswith("TCC_") else 0) for n in names)
            assert tcc <= 4, line
            assert sum(n.startswith("SQ_") for n in names) <= 8, line
            assert all(re.fullmatch(r"[A-Z][A-Za-z0-9_]*", n) for n in names), line
