"""CPU float64 oracle for the distributed Operator Inference (dOpInf) hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
(``paper_2504_14338_amd``) never imports, links or calls anything here, and
nothing here imports the product.

Every function is plain, slow and written to be checked against the paper by
eye: float64 numpy, library primitives (matmul, eigh, solve, cholesky) used as
single steps, explicit Python loops where the paper's steps are loops.  Each
function cites the section / equation of arXiv:2504.14338 it follows.

Conventions (as in the paper's listings): Q is n x k (rows = degrees of
freedom, columns = snapshots); each state variable is a contiguous block of
rows ``var_rows[v]:var_rows[v+1]``; reduced data Qhat is r x k.

Readings where the paper is silent or inconsistent are marked READING and
listed in the design notes of the repository.
"""
from __future__ import annotations

import numpy as np

from .pipeline import *  # noqa: F401,F403
from .pipeline import __all__  # noqa: F401
from . import continuous  # noqa: F401
