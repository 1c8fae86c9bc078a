"""MI355X-native Background SHAP for decision-tree ensembles (WOODELF hot path)."""
