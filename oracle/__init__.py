"""CPU oracle for the chemistry hot path.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2105_12070_amd``) never imports it, and the two share no code; only
the seeded input generator feeds both.
"""
from .oracle import *  # noqa: F401,F403
