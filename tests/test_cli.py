"""The command-line entry points parse their arguments without a GPU
(--help exits 0 before any device work; a bad choice exits 2)."""
import pytest


@pytest.mark.parametrize("module", ["solve", "batched", "learned"])
def test_cli_help(module, capsys):
    import importlib
    mod = importlib.import_module(f"paper_1505_08023_amd.{module}")
    with pytest.raises(SystemExit) as e:
        mod.main(["--help"])
    assert e.value.code == 0
    assert "usage" in capsys.readouterr().out


def test_cli_rejects_unknown_method():
    from paper_1505_08023_amd import solve
    with pytest.raises(SystemExit) as e:
        solve.main(["--method", "gmres"])
    assert e.value.code == 2
