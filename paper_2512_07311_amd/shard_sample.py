"""One independent sampling job (Section 3.2, stage 3): load a persisted
state, draw shots [first, first + count) with the given seed on this
process's GPU, and write the bitstrings (uint64) and their log2
probabilities (float64) to an .npz file.

Jobs over disjoint ranges of the same state and seed merge, by
concatenation in shot order, into exactly the shots one call over the
whole range draws: each shot depends only on the state, the seed and its
index.

Usage: python -m paper_2512_07311_amd.shard_sample STATE FIRST COUNT SEED OUT.npz
"""
import sys


def main(argv):
    if len(argv) != 5:
        print(__doc__, file=sys.stderr)
        return 2
    path, first, count, seed, out = argv[0], int(argv[1]), int(argv[2]), int(argv[3]), argv[4]
    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("shard_sample needs a GPU", file=sys.stderr)
        return 1
    import paper_2512_07311_amd as rcs
    torch.cuda.set_device(0)
    st = rcs.State.load(path)
    bits = torch.zeros(count, dtype=torch.int64, device="cuda")
    l2 = torch.zeros(count, dtype=torch.float64, device="cuda")
    st.sample(bits, l2, seed=seed, first_shot=first)
    torch.cuda.synchronize()
    np.savez(out, bits=bits.cpu().numpy().view(np.uint64), log2p=l2.cpu().numpy(),
             first=np.int64(first), seed=np.uint64(seed))
    print("shard_sample: %d shots from %d written to %s" % (count, first, out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
