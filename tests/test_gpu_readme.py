"""The README's quick start, run as written: the documented calls work
together and give a positive, finite scatter estimate."""
import os
import re

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_quick_start_runs():
    text = open(os.path.join(ROOT, "README.md")).read()
    code = re.search(r"## Quick start \(Python\)\n\n```python\n(.*?)```", text, re.S).group(1)
    env = {}
    exec(compile(code, "README.md quick start", "exec"), env)
    torch.cuda.synchronize()
    est, out, ctx = env["est"], env["out"], env["ctx"]
    try:
        assert int(out["scatter_counts"].sum()) > 1_000_000
        assert bool(torch.isfinite(est).all()) and float(est.min()) >= 0.0 and float(est.sum()) > 0.0
    finally:
        ctx.close()
