"""pic_mlp_forward_static, the network's forward pass for callers that
cannot allocate (its BF16 weights and hidden activations in the library's
fixed device array instead of a workspace), against pic_mlp_forward on the
same parameters and inputs: the same kernels on the same operands, so the
outputs must be equal bit for bit. Two calls in a row, the second with a
smaller network and batch, then the first shape again; a call beyond the
array's size is refused before anything runs."""
import numpy as np
import pytest

from gpu_common import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _params(dims, rng):
    n_in, width, depth, n_out = dims
    sizes = [n_in] + [width] * depth + [n_out]
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        parts.append(rng.normal(scale=np.sqrt(2.0 / a), size=a * b))
        parts.append(rng.normal(scale=0.1, size=b))
    return np.concatenate(parts).astype(np.float32)


def test_static_forward_equals_workspace_forward():
    import torch

    from paper_2109_04469_amd import Mlp, PicError, mlp_forward_static

    dev = torch.device("cuda:0")
    cases = [((6, 256, 4, 512), 300, 1), ((6, 64, 2, 128), 7, 2), ((6, 256, 4, 512), 1000, 3)]
    for k, (dims, batch, seed) in enumerate(cases):
        print(f"[no-alloc] call {k}: dims {dims} batch {batch}", flush=True)
        rng = np.random.default_rng(seed)
        p = _params(dims, rng)
        net = Mlp(*dims, max_batch=batch)
        assert net.num_params == p.size
        net.set_params(p)
        x = rng.uniform(-1.0, 1.0, (batch, dims[0])).astype(np.float32)
        ref = net.forward(x).cpu().numpy()
        got = mlp_forward_static(dims, torch.as_tensor(p, device=dev), torch.as_tensor(x, device=dev))
        got = got.cpu().numpy()
        assert got.shape == ref.shape
        assert np.array_equal(got, ref), f"call {k}: max diff {np.max(np.abs(got - ref))}"
        net.close()
    # beyond the fixed array (3000 rows of 256 activations): refused
    dims = (6, 256, 4, 512)
    p = torch.as_tensor(_params(dims, np.random.default_rng(4)), device=dev)
    with pytest.raises(PicError):
        mlp_forward_static(dims, p, torch.zeros((3000, 6), dtype=torch.float32, device=dev))
    # bad shapes are refused too
    with pytest.raises(PicError):
        mlp_forward_static((0, 256, 4, 512), p, torch.zeros((4, 6), dtype=torch.float32, device=dev))
