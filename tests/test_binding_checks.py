"""The binding refuses a device buffer of the wrong kind before its address
reaches the library (no GPU needed): the library reads or writes exactly N
records through each pointer, so a float32 state, a transposed tensor, a short
output or a host tensor would otherwise reach device memory out of bounds."""
import pytest
import torch

import paper_2208_13770_amd as vb

N = 10


@pytest.fixture
def fake_ctx(monkeypatch):
    """A context of N particles as far as the shape checks can tell; any call that
    got past the checks into the library would fail on the None context."""
    monkeypatch.setattr(vb, "vb_get_info",
                        lambda ctx: {"n_total": N, "n_sys": 1, "row_width": 32, "step": 0})
    return None


def state(dtype_x=torch.float64, dtype_r=torch.float32, n=N):
    return (torch.zeros(n, 3, dtype=dtype_x), torch.zeros(n, 3, dtype=dtype_x),
            torch.ones(n, dtype=dtype_r), torch.ones(n, dtype=dtype_r))


def test_set_state_refuses_wrong_dtype(fake_ctx):
    x, v, rc, invm = state(dtype_x=torch.float32)
    with pytest.raises(ValueError, match="x must be torch.float64"):
        vb.vb_set_state(fake_ctx, x, v, rc, invm)
    x, v, rc, invm = state(dtype_r=torch.float64)
    with pytest.raises(ValueError, match="rc must be torch.float32"):
        vb.vb_set_state(fake_ctx, x, v, rc, invm)


def test_set_state_refuses_non_contiguous_and_short_buffers(fake_ctx):
    x, v, rc, invm = state()
    with pytest.raises(ValueError, match="contiguous"):
        vb.vb_set_state(fake_ctx, torch.zeros(3, N, dtype=torch.float64).t(), v, rc, invm)
    with pytest.raises(ValueError, match=r"shape \[10, 3\]"):
        vb.vb_set_state(fake_ctx, x[:N - 1], v, rc, invm)
    with pytest.raises(ValueError, match=r"invm must have shape \[10\]"):
        vb.vb_set_state(fake_ctx, x, v, rc, invm[:N - 2])


def test_set_state_refuses_host_tensors(fake_ctx):
    x, v, rc, invm = state()
    with pytest.raises(ValueError, match="GPU tensor"):
        vb.vb_set_state(fake_ctx, x, v, rc, invm)
    with pytest.raises(ValueError, match="torch tensor"):
        vb.vb_set_state(fake_ctx, x.numpy(), v, rc, invm)


def test_get_state_refuses_wrong_outputs(fake_ctx):
    with pytest.raises(ValueError, match="float64"):
        vb.vb_get_state(fake_ctx, torch.zeros(N, 3, dtype=torch.float32))
    with pytest.raises(ValueError, match="shape"):
        vb.vb_get_state(fake_ctx, None, torch.zeros(N + 1, 3, dtype=torch.float64))


def test_get_pairs_refuses_short_delta_and_wrong_dtype(fake_ctx):
    pairs = torch.zeros(8, 2, dtype=torch.int32)
    with pytest.raises(ValueError, match=r"delta must have shape \[8\]"):
        vb.vb_get_pairs(fake_ctx, 0, 0, pairs, torch.zeros(7, dtype=torch.float64))
    with pytest.raises(ValueError, match="int32"):
        vb.vb_get_pairs(fake_ctx, 0, 0, torch.zeros(8, 2, dtype=torch.int64))
    with pytest.raises(ValueError, match=r"\[cap, 2\]"):
        vb.vb_get_pairs(fake_ctx, 0, 0, torch.zeros(16, dtype=torch.int32))
    with pytest.raises(ValueError, match="delta needs pairs"):
        vb.vb_get_pairs(fake_ctx, 0, 0, None, torch.zeros(8, dtype=torch.float64))


def test_history_refuses_mismatched_tables(fake_ctx):
    partner = torch.zeros(N, 4, dtype=torch.int32)
    with pytest.raises(ValueError, match=r"spring must have shape \[10, 4, 3\]"):
        vb.vb_set_history(fake_ctx, partner, torch.zeros(N, 3, 3, dtype=torch.float64))
    with pytest.raises(ValueError, match=r"partner must have shape \[10, 4\]"):
        vb.vb_get_history(fake_ctx, partner[:5], torch.zeros(5, 4, 3, dtype=torch.float64))
    with pytest.raises(ValueError, match="go together"):
        vb.vb_set_history(fake_ctx, partner, None)
