"""GPU: the usage example of the README runs as written, scaled down (R = 2000,
50 MD steps per temperature), and ends at T_final with a consistent
population."""
import os
import re

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    text = open(os.path.join(ROOT, "README.md")).read()
    code = re.search(r"```python\n(.*?)```", text, re.S).group(1)
    assert "R_target=100_000" in code and "md_steps(1000)" in code
    code = code.replace("R_target=100_000", "R_target=2000").replace("md_steps(1000)", "md_steps(50)")
    ns = {}
    exec(compile(code, "README example", "exec"), ns)
    obs = ns["obs"]
    print({k: obs[k] for k in ("T", "temp_index", "R", "families", "sum_lnQ")})
    assert obs["T"] == 250.0 and obs["temp_index"] > 5
    assert 1 <= obs["families"] <= obs["R"] and abs(obs["R"] - 2000) < 200
    assert obs["sum_lnQ"] != 0.0
