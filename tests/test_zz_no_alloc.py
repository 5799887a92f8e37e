"""The backward pass without allocation (trajam_mlp_backward_noalloc) against the
backward pass with a caller workspace (trajam_mlp_backward), through the C ABI: the
same kernels on the same inputs, so every gradient must be bitwise equal.  Two calls
in a row, the second with a smaller batch (the static workspace keeps the first
call's contents), in both precisions; a request beyond the workspace is rejected
on the host."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(tj, widths, batch, precision, seed):
    rng = np.random.default_rng(seed)
    shape = tj.mlp_shape(widths)
    n = tj.trajam_mlp_param_count(shape)
    params = torch.as_tensor(rng.normal(size=n) * 0.1, dtype=torch.float32, device="cuda")
    x = torch.as_tensor(rng.normal(size=(batch, widths[0])), dtype=torch.float32, device="cuda")
    hid = sum(widths[1:-1])
    acts = torch.zeros(max(hid, 1) * batch, device="cuda")
    y = torch.zeros((batch, widths[-1]), device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    tj.trajam_mlp_forward(shape, batch, precision, params.data_ptr(), x.data_ptr(), acts.data_ptr(),
                          y.data_ptr(), st)
    dy = torch.as_tensor(rng.normal(size=(batch, widths[-1])), dtype=torch.float32, device="cuda")
    maxw = max(widths[1:-1])
    ws = torch.zeros(2 * batch * maxw, device="cuda")
    g_ref = torch.full((n,), float("nan"), device="cuda")
    g_new = torch.full((n,), float("nan"), device="cuda")
    tj.trajam_mlp_backward(shape, batch, precision, params.data_ptr(), x.data_ptr(), acts.data_ptr(),
                           dy.data_ptr(), g_ref.data_ptr(), ws.data_ptr(), st)
    tj.trajam_mlp_backward_noalloc(shape, batch, precision, params.data_ptr(), x.data_ptr(),
                                   acts.data_ptr(), dy.data_ptr(), g_new.data_ptr(), st)
    torch.cuda.synchronize()
    return g_ref.cpu().numpy(), g_new.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_backward_equals_backward_on_two_calls(precision):
    from paper_2408_10731_amd import trajam as tj
    for widths, batch in (([44, 256, 256, 22], 1024), ([44, 256, 256, 22], 37)):
        print(f"case: mlp backward noalloc, widths {widths}, batch {batch}, precision {precision}",
              flush=True)
        ref, new = _case(tj, widths, batch, precision, seed=batch + precision)
        assert np.all(np.isfinite(ref))
        assert np.array_equal(ref, new)


def test_noalloc_backward_rejects_oversized_batch():
    from paper_2408_10731_amd import trajam as tj
    widths = [8, 512, 4]
    batch = tj.MLP_NOALLOC_SCRATCH_FLOATS // (2 * 512) + 1
    shape = tj.mlp_shape(widths)
    with pytest.raises(tj.TrajamError) as e:
        # rejected on the host before any pointer is touched
        tj.trajam_mlp_backward_noalloc(shape, batch, 0, 1, 1, 1, 1, 1, None)
    assert e.value.status == tj.TRAJAM_ERR_CAPACITY
