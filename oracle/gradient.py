"""d ln L / d lambda (TEST INFRASTRUCTURE; see package header).

Central finite differences of likelihood.lnl; the analytic chain rule is
added beside it.
"""
