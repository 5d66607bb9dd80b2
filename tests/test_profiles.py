"""The rocprofv3 summaries under profiles/: each gives the full command that made it, and
that command runs a file of this repository (never a scratch script)."""
import pathlib
import re

ROOT = pathlib.Path(__file__).resolve().parent.parent


def _summaries():
    return sorted((ROOT / "profiles").glob("*.md"))


def test_there_are_summaries():
    assert _summaries()


def test_each_summary_names_a_committed_program():
    for f in _summaries():
        text = f.read_text()
        cmds = [ln for ln in text.splitlines() if ln.startswith("rocprofv3 ")]
        assert cmds, f.name
        for c in cmds:
            assert " -- " in c, (f.name, c)
            prog = c.split(" -- ", 1)[1].split()
            assert prog[0] in ("python3", "python"), (f.name, c)
            m = re.match(r"\$GRAFT_REPO_ROOT/(.+)", prog[1])
            assert m, (f.name, prog[1])
            path = m.group(1)
            assert not path.startswith("_work"), (f.name, path)
            assert (ROOT / path).is_file(), (f.name, path)
            assert "--pmc" not in c or not re.search(r"(^| )(-s|-r|--sys-trace|--runtime-trace)( |$)", c)
