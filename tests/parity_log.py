"""Per-class parity lines collected during a test session.

The GPU parity tests record one line per comparison (status agreement and
the class sizes and maxima of the flow differences); the session's terminal
summary prints them, so they reach the log under -q as well.
"""
LINES = []


def record(line: str) -> None:
    LINES.append(line)
    print(line)
