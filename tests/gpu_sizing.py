"""Largest cubic lattice the free device memory holds, for the maximum-size
GPU tests."""


def largest_edge(torch, precision, lo=256, hi=488, step=8, extra_per_site=16 * 9, margin=6 << 30):
    """Edge (lo..hi in steps of `step`) of the largest cubic lattice of the
    given precision whose buffers fit the free device memory beside
    `extra_per_site` bytes per site (an FP64 moments array and change) and a
    margin."""
    from paper_1505_02037_amd import lb

    torch.cuda.empty_cache()  # memory torch cached for earlier tests counts as free here
    free, _ = torch.cuda.mem_get_info()
    e = lo
    while e < hi:
        nxt = e + step
        need = lb.device_bytes(nxt, nxt, nxt, precision=precision) + extra_per_site * nxt ** 3 + margin
        if need > free:
            break
        e = nxt
    return e
