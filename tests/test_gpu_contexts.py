"""Contexts on one device share the MT19937 tables: the second context's
first MT19937 call builds nothing (no new device memory for the 656 MB of
tables), results agree across contexts and with the oracle, and the tables
stay valid until the last context that holds them is destroyed."""
import numpy as np
import pytest
import torch

from paper_1307_5869_amd import prand as P

pytestmark = pytest.mark.gpu

SID = 2**63 + 12345


def test_mt19937_tables_shared_across_contexts(oracle):
    ref = oracle.init_stream(P.MT19937, P.SEQ_DEFAULT, SID)
    a = P.Context(0)
    b = P.Context(0)
    sa = a.init_stream(P.MT19937, P.SEQ_DEFAULT, SID)   # builds the tables, or shares an older context's
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    sb = b.init_stream(P.MT19937, P.SEQ_DEFAULT, SID)   # shares them
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < (64 << 20), (free0, free1)
    assert np.array_equal(sa, ref) and np.array_equal(sb, ref)
    a.close()
    # the tables outlive the context that built them
    assert np.array_equal(b.init_stream(P.MT19937, P.SEQ_DEFAULT, SID), ref)
    ids = torch.tensor(np.array([0, 7, SID, 2**64 - 1], dtype=np.uint64).view(np.int64), device="cuda")
    d = torch.empty(4 * P.state_bytes(P.MT19937), dtype=torch.uint8, device="cuda")
    b.init_streams_dev(P.MT19937, P.SEQ_DEFAULT, None, ids, 4, d)
    torch.cuda.synchronize()
    got_b = d.cpu().numpy().copy()
    b.close()
    # a context made after every earlier holder is gone builds them again
    c = P.Context(0)
    d.zero_()
    c.init_streams_dev(P.MT19937, P.SEQ_DEFAULT, None, ids, 4, d)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), got_b)
    assert np.array_equal(got_b[2 * P.state_bytes(P.MT19937):3 * P.state_bytes(P.MT19937)], ref)
    c.close()
