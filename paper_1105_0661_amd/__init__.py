"""lbf: an MI355X-native tied-array beam former (Mol & Romein, arxiv 1105.0661)."""
